// Dispatch to the compile-time-radius kernels (bsk_radius.h): which launches
// have them, and the part file that holds the radius.
#include "bsk_radius.h"

namespace bsk {

namespace {

bool radius_ct(int block, int rh) { return block == 256 && rh >= 1 && rh <= kRadiusCtMax; }
bool radius_ct_bwd(int block, int rh) { return block == 256 && rh >= 1 && rh <= kRadiusCtMaxBwd; }

}  // namespace

bool forward_radius_kernel(int block, int rh) { return radius_ct(block, rh); }
bool train_radius_kernel(int block, int rh) { return radius_ct(block, rh); }
bool backward_radius_kernel(int block, int rh, int kc)
{
    return radius_ct_bwd(block, rh) && (kc == 24 || kc == 16 || kc == 8);
}

hipError_t launch_forward_f32_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    static_assert(kRadiusCtMax == 8 * kRadiusPerPart, "eight parts of radii");
    if (!radius_ct(256, a.rh)) return hipErrorInvalidValue;
    switch ((a.rh - 1) / kRadiusPerPart) {
    case 0: return forward_radius_1_8(a, kc, s, occ);
    case 1: return forward_radius_9_16(a, kc, s, occ);
    case 2: return forward_radius_17_24(a, kc, s, occ);
    case 3: return forward_radius_25_32(a, kc, s, occ);
    case 4: return forward_radius_33_40(a, kc, s, occ);
    case 5: return forward_radius_41_48(a, kc, s, occ);
    case 6: return forward_radius_49_56(a, kc, s, occ);
    default: return forward_radius_57_64(a, kc, s, occ);
    }
}

hipError_t launch_train_f32_radius(const StripArgs &a, hipStream_t s, int *occ)
{
    if (!radius_ct(256, a.rh)) return hipErrorInvalidValue;
    switch ((a.rh - 1) / kRadiusPerPart) {
    case 0: return train_radius_1_8(a, s, occ);
    case 1: return train_radius_9_16(a, s, occ);
    case 2: return train_radius_17_24(a, s, occ);
    case 3: return train_radius_25_32(a, s, occ);
    case 4: return train_radius_33_40(a, s, occ);
    case 5: return train_radius_41_48(a, s, occ);
    case 6: return train_radius_49_56(a, s, occ);
    default: return train_radius_57_64(a, s, occ);
    }
}

hipError_t launch_backward_f32_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    static_assert(kRadiusCtMaxBwd == 4 * kRadiusPerPart, "four parts of adjoint radii");
    if (!radius_ct_bwd(256, a.rh)) return hipErrorInvalidValue;
    switch ((a.rh - 1) / kRadiusPerPart) {
    case 0: return backward_radius_1_8(a, kc, s, occ);
    case 1: return backward_radius_9_16(a, kc, s, occ);
    case 2: return backward_radius_17_24(a, kc, s, occ);
    default: return backward_radius_25_32(a, kc, s, occ);
    }
}

}  // namespace bsk
