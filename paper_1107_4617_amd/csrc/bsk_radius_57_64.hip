// Compile-time-radius forward and training-forward kernels for the
// radii 57 to 64 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_57_64(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<57>(a, kc, s, occ);
}
hipError_t train_radius_57_64(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<57>(a, s, occ); }

}  // namespace bsk
