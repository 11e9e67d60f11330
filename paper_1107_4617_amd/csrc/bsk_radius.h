// The 256-lane plain FP32 forward and training forward (every radius 1 to 64,
// all that 256-lane strips take by default) and adjoint (radii 1 to 32) with
// the box radius as a compile-time constant.  Their walkers
// hand box sums to the R stage instead of prefix sums (strip_body, RHC > 0),
// which halves the R stage's LDS reads: the forward's R stage reads four
// channels per order, the training forward's six and the adjoint's four.
// Other radii, the 16-bit and compensated stacks use the run-time-radius
// kernels of bsk_kernels.hip.
//
// The radii are compiled in eight parts of eight (bsk_radius_1_8.hip ...
// bsk_radius_57_64.hip), so the build compiles them in parallel; bsk_radius.hip
// picks the part.
#pragma once
#include <utility>

#include "bsk_strip.h"

namespace bsk {

constexpr int kRadiusCtMax = 64;      // forward and training forward: radii 1 .. kRadiusCtMax
// The adjoint's: above 32 the run-time-radius adjoint, with its one-pass
// kernels' constant start mode, measured as fast (0.675 ms at r = 40, 4096^2).
constexpr int kRadiusCtMaxBwd = 32;
constexpr int kRadiusPerPart = 8;

// One pass with the start mode as a constant (K <= KR), else passes with the
// run-time mode.
template <int R, int KR>
hipError_t fwd_radius_pass(const StripArgs &a, hipStream_t s, int *occ)
{
    constexpr int KL = kl_f32(256);
    if (a.K <= KR && a.start_mode == 0) return launch<float, 256, KR, KL, PolForward<float, 0>, 0, false, 3, R>(a, s, occ);
    if (a.K <= KR && a.start_mode == 1) return launch<float, 256, KR, KL, PolForward<float, 1>, 0, false, 3, R>(a, s, occ);
    return launch<float, 256, KR, KL, PolForward<float>, 0, false, 3, R>(a, s, occ);
}

// The pass sizes of the 256-lane plain FP32 forward: 8, 12, 16, 20 and 24 orders.
template <int R>
hipError_t fwd_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    static_assert(kr_f32(256) == 16 && kl_f32(256) == 4, "the pass sizes below are the 256-lane ones");
    switch (kc) {
    case 24: return fwd_radius_pass<R, 24>(a, s, occ);
    case 20: return fwd_radius_pass<R, 20>(a, s, occ);
    case 16: return fwd_radius_pass<R, 16>(a, s, occ);
    case 12: return fwd_radius_pass<R, 12>(a, s, occ);
    case 8: return fwd_radius_pass<R, 8>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}

// The training forward's 8-order pass; one-pass launches take the start mode as
// a constant.  (A single 16-order pass, at two workgroups per CU, measured 11%
// slower than two 8-order passes at three.)
template <int R>
hipError_t train_radius(const StripArgs &a, hipStream_t s, int *occ)
{
    constexpr int KR = kr_train(256), KL = kl_train(256);
    if (a.K <= KR && a.start_mode == 0) return launch<float, 256, KR, KL, PolTrain<0>, 0, false, 3, R>(a, s, occ);
    if (a.K <= KR && a.start_mode == 1) return launch<float, 256, KR, KL, PolTrain<1>, 0, false, 3, R>(a, s, occ);
    return launch<float, 256, KR, KL, PolTrain<>, 0, false, 3, R>(a, s, occ);
}

template <int R, int KR, int MINB>
hipError_t backward_radius_pass(const StripArgs &a, hipStream_t s, int *occ)
{
    if (a.K <= KR && a.start_mode == 0) return bwd<256, KR, 4, MINB, R, 0>(a, s, occ);
    if (a.K <= KR && a.start_mode == 1) return bwd<256, KR, 4, MINB, R, 1>(a, s, occ);
    return bwd<256, KR, 4, MINB, R>(a, s, occ);
}

// The adjoint's pass shapes at 256 lanes: 24 orders at two workgroups per CU,
// 16 orders (three per CU in one pass with the start mode as a constant, two
// otherwise), the 8-order half pass at three.
template <int R>
hipError_t backward_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    switch (kc) {
    case 24: return backward_radius_pass<R, 24, 2>(a, s, occ);
    case 16: return backward_radius_pass<R, 16, 0>(a, s, occ);
    case 8: return bwd<256, 8, 4, 3, R>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}

// Calls f(std::integral_constant<int, R>) for the R in LO .. LO + N - 1 that
// equals r; hipErrorInvalidValue when none does.
template <int LO, class F, int... I>
hipError_t with_radius(int r, F &&f, std::integer_sequence<int, I...>)
{
    hipError_t e = hipErrorInvalidValue;
    (void)((r == LO + I ? (e = f(std::integral_constant<int, LO + I>{}), true) : false) || ...);
    return e;
}

// Radii LO .. LO + kRadiusPerPart - 1 of each kernel family; each part file
// instantiates one LO.
template <int LO>
hipError_t forward_radii(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return with_radius<LO>(a.rh, [&](auto R) { return fwd_radius<decltype(R)::value>(a, kc, s, occ); },
                           std::make_integer_sequence<int, kRadiusPerPart>{});
}
template <int LO>
hipError_t train_radii(const StripArgs &a, hipStream_t s, int *occ)
{
    return with_radius<LO>(a.rh, [&](auto R) { return train_radius<decltype(R)::value>(a, s, occ); },
                           std::make_integer_sequence<int, kRadiusPerPart>{});
}
template <int LO>
hipError_t backward_radii(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    return with_radius<LO>(a.rh, [&](auto R) { return backward_radius<decltype(R)::value>(a, kc, s, occ); },
                           std::make_integer_sequence<int, kRadiusPerPart>{});
}

// The part files' entry points (radii 1-8, 9-16, 17-24, 25-32: all three families).
#define BSK_RADIUS_PART_DECL(LO, HI)                                                                    \
    hipError_t forward_radius_##LO##_##HI(const StripArgs &a, int kc, hipStream_t s, int *occ);          \
    hipError_t train_radius_##LO##_##HI(const StripArgs &a, hipStream_t s, int *occ);                    \
    hipError_t backward_radius_##LO##_##HI(const StripArgs &a, int kc, hipStream_t s, int *occ);
BSK_RADIUS_PART_DECL(1, 8)
BSK_RADIUS_PART_DECL(9, 16)
BSK_RADIUS_PART_DECL(17, 24)
BSK_RADIUS_PART_DECL(25, 32)
#undef BSK_RADIUS_PART_DECL
// forward and training forward only
#define BSK_RADIUS_PART_DECL_FT(LO, HI)                                                                 \
    hipError_t forward_radius_##LO##_##HI(const StripArgs &a, int kc, hipStream_t s, int *occ);          \
    hipError_t train_radius_##LO##_##HI(const StripArgs &a, hipStream_t s, int *occ);
BSK_RADIUS_PART_DECL_FT(33, 40)
BSK_RADIUS_PART_DECL_FT(41, 48)
BSK_RADIUS_PART_DECL_FT(49, 56)
BSK_RADIUS_PART_DECL_FT(57, 64)
#undef BSK_RADIUS_PART_DECL_FT

}  // namespace bsk
