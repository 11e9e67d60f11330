// Compile-time-radius forward, training-forward and adjoint kernels for the
// radii 1 to 8 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_1_8(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<1>(a, kc, s, occ);
}
hipError_t train_radius_1_8(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<1>(a, s, occ); }
hipError_t backward_radius_1_8(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return backward_radii<1>(a, kc, s, occ);
}

}  // namespace bsk
