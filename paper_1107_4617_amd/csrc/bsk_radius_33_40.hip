// Compile-time-radius forward and training-forward kernels for the
// radii 33 to 40 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_33_40(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<33>(a, kc, s, occ);
}
hipError_t train_radius_33_40(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<33>(a, s, occ); }

}  // namespace bsk
