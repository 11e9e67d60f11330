// Two-pixel-patch kernels (256 lanes, 16-order pass, every packing) with the
// box radius as a compile-time constant, at the radii 3, 5, 8, 10, 16, 20, 25
// and 32: their walkers hand box sums to the R stage instead of prefix sums
// (strip_body, RHC > 0), which halves the R stage's LDS reads.  Other radii
// and the half pass use the run-time-radius kernels of bsk_kernels.hip.
#include "bsk_strip.h"

namespace bsk {

namespace {

static_assert(kr_f32(256) == kPatchPackPass, "the patch kernels use the 256-lane full pass");

// packing G (0: unpacked, one group per pass)
template <int R, int G = kPatchPackMax>
hipError_t patch_radius(const StripArgs &a, int pack, hipStream_t s, int *occ)
{
    if (pack == G) return launch<float, 256, kPatchPackPass, kl_f32(256), PolPatch2G<G>, 0, false, 3, R>(a, s, occ);
    if constexpr (G > 0) return patch_radius<R, G - 1>(a, pack, s, occ);
    return hipErrorInvalidValue;
}

}  // namespace

bool patch_radius_kernel(int block, int kc, int rh)
{
    if (block != 256 || kc != kPatchPackPass) return false;
    switch (rh) {
    case 3: case 5: case 8: case 10: case 16: case 20: case 25: case 32: return true;
    default: return false;
    }
}

hipError_t launch_patch2_f32_radius(const StripArgs &a, int pack, hipStream_t s, int *occ)
{
    switch (a.rh) {
    case 3: return patch_radius<3>(a, pack, s, occ);
    case 5: return patch_radius<5>(a, pack, s, occ);
    case 8: return patch_radius<8>(a, pack, s, occ);
    case 10: return patch_radius<10>(a, pack, s, occ);
    case 16: return patch_radius<16>(a, pack, s, occ);
    case 20: return patch_radius<20>(a, pack, s, occ);
    case 25: return patch_radius<25>(a, pack, s, occ);
    case 32: return patch_radius<32>(a, pack, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bsk
