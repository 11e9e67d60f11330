// Compile-time-radius forward and training-forward kernels for the
// radii 49 to 56 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_49_56(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<49>(a, kc, s, occ);
}
hipError_t train_radius_49_56(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<49>(a, s, occ); }

}  // namespace bsk
