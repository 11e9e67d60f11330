// One-pass plain FP32 forward (256 lanes, the full and the half pass) with
// the box radius as a compile-time constant, for a set of common radii.  Its
// walkers hand box sums to the R stage instead of prefix sums (strip_body,
// RHC > 0), which halves the R stage's LDS reads.  Other radii, and every
// other form, use the run-time-radius kernels of bsk_kernels.hip.
#include "bsk_strip.h"

namespace bsk {

namespace {

template <int R>
hipError_t fwd_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    constexpr int KR = kr_f32(256), KL = kl_f32(256);
    if (kc == KR)
        return a.start_mode == 0 ? launch<float, 256, KR, KL, PolForward<float, 0>, 0, false, 3, R>(a, s, occ)
                                 : launch<float, 256, KR, KL, PolForward<float, 1>, 0, false, 3, R>(a, s, occ);
    return a.start_mode == 0 ? launch<float, 256, KR / 2, KL, PolForward<float, 0>, 0, false, 3, R>(a, s, occ)
                             : launch<float, 256, KR / 2, KL, PolForward<float, 1>, 0, false, 3, R>(a, s, occ);
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
    if ((kc != kr_f32(256) && kc != kr_f32(256) / 2) || a.K > kc || (a.start_mode != 0 && a.start_mode != 1))
        return hipErrorInvalidValue;
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
