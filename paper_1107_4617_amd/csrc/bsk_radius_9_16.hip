// Compile-time-radius forward, training-forward and adjoint kernels for the
// radii 9 to 16 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_9_16(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<9>(a, kc, s, occ);
}
hipError_t train_radius_9_16(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<9>(a, s, occ); }
hipError_t backward_radius_9_16(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return backward_radii<9>(a, kc, s, occ);
}

}  // namespace bsk
