// Compile-time-radius forward, training-forward and adjoint kernels for the
// radii 17 to 24 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_17_24(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<17>(a, kc, s, occ);
}
hipError_t train_radius_17_24(const StripArgs &a, hipStream_t s, int *occ) { return train_radii<17>(a, s, occ); }
hipError_t backward_radius_17_24(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return backward_radii<17>(a, kc, s, occ);
}

}  // namespace bsk
