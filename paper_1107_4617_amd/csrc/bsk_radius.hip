// Plain FP32 forward (256 lanes, passes of 16, 12 or 8 orders, one pass or
// several) with the box radius as a compile-time constant, for a set of
// common radii.  Its walkers hand box sums to the R stage instead of prefix
// sums (strip_body, RHC > 0), which halves the R stage's LDS reads.  Other
// radii, and the 16-bit and compensated stacks, use the run-time-radius
// kernels of bsk_kernels.hip.
#include "bsk_strip.h"

namespace bsk {

namespace {

template <int R, int KR>
hipError_t fwd_radius_pass(const StripArgs &a, hipStream_t s, int *occ)
{
    constexpr int KL = kl_f32(256);
    // one pass with the start mode as a constant, else passes with the run-time mode
    if (a.K <= KR && a.start_mode == 0) return launch<float, 256, KR, KL, PolForward<float, 0>, 0, false, 3, R>(a, s, occ);
    if (a.K <= KR && a.start_mode == 1) return launch<float, 256, KR, KL, PolForward<float, 1>, 0, false, 3, R>(a, s, occ);
    return launch<float, 256, KR, KL, PolForward<float>, 0, false, 3, R>(a, s, occ);
}

// the three pass sizes of the 256-lane plain FP32 forward: 16, 12 and 8 orders
template <int R>
hipError_t fwd_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    switch (kc) {
    case 16: return fwd_radius_pass<R, 16>(a, s, occ);
    case 12: return fwd_radius_pass<R, 12>(a, s, occ);
    case 8: return fwd_radius_pass<R, 8>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool forward_radius_kernel(int block, int rh)
{
    if (block != 256) return false;
    switch (rh) {
    case 3: case 5: case 8: case 10: case 16: case 20: case 25: case 32: return true;
    default: return false;
    }
}

hipError_t launch_forward_f32_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    static_assert(kr_f32(256) == 16 && kl_f32(256) == 4, "the pass sizes below are the 256-lane ones");
    switch (a.rh) {
    case 3: return fwd_radius<3>(a, kc, s, occ);
    case 5: return fwd_radius<5>(a, kc, s, occ);
    case 8: return fwd_radius<8>(a, kc, s, occ);
    case 10: return fwd_radius<10>(a, kc, s, occ);
    case 16: return fwd_radius<16>(a, kc, s, occ);
    case 20: return fwd_radius<20>(a, kc, s, occ);
    case 25: return fwd_radius<25>(a, kc, s, occ);
    case 32: return fwd_radius<32>(a, kc, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bsk
