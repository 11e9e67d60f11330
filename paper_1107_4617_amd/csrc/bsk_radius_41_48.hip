// Compile-time-radius forward and training-forward kernels for the
// radii 41 to 48 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_41_48(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<41>(a, kc, s, occ);
}
hipError_t train_radius_41_48(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<41>(a, s, occ); }

}  // namespace bsk
