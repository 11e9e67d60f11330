// Compile-time-radius forward kernels for the radii 41 to 48 (bsk_radius.h).
#include "bsk_radius.h"

namespace bsk {

hipError_t forward_radius_41_48(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return forward_radii<41>(a, kc, s, occ);
}

}  // namespace bsk
