// Compile-time-radius forward, training-forward and adjoint kernels for the
// radii 25 to 32 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_25_32(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<25>(a, kc, s, occ);
}
hipError_t train_radius_25_32(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<25>(a, s, occ); }
hipError_t backward_radius_25_32(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return backward_radii<25>(a, kc, s, occ);
}

}  // namespace bsk
