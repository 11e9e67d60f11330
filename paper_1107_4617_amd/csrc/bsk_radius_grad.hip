// Training forward and adjoint (256 lanes) with the box radius as a
// compile-time constant, for the radii that have compile-time-radius forward
// kernels (bsk_radius.hip).  Their walkers hand box sums to the R stage, which
// then reads one value per channel instead of two: the training forward's R
// stage reads six channels per order and the adjoint's four, so both gain more
// than the forward.  Other radii use the run-time-radius kernels.
#include "bsk_strip.h"

namespace bsk {

namespace {

template <int R>
hipError_t train_radius(const StripArgs &a, hipStream_t s, int *occ)
{
    constexpr int KR = kr_train(256), KL = kl_train(256);
    // one pass with the start mode as a constant, else passes with the run-time
    // mode (a single 16-order pass, at two workgroups per CU, measured 11%
    // slower than two 8-order passes at three)
    if (a.K <= KR && a.start_mode == 0) return launch<float, 256, KR, KL, PolTrain<0>, 0, false, 3, R>(a, s, occ);
    if (a.K <= KR && a.start_mode == 1) return launch<float, 256, KR, KL, PolTrain<1>, 0, false, 3, R>(a, s, occ);
    return launch<float, 256, KR, KL, PolTrain<>, 0, false, 3, R>(a, s, occ);
}

// one pass with the start mode as a constant, else passes with the run-time mode
template <int R, int KR, int MINB>
hipError_t backward_radius_pass(const StripArgs &a, hipStream_t s, int *occ)
{
    if (a.K <= KR && a.start_mode == 0) return bwd<256, KR, 4, MINB, R, 0>(a, s, occ);
    if (a.K <= KR && a.start_mode == 1) return bwd<256, KR, 4, MINB, R, 1>(a, s, occ);
    return bwd<256, KR, 4, MINB, R>(a, s, occ);
}

// the pass shapes of bwd_block<256>: the 24- and 16-order passes at two
// workgroups per CU, the 8-order half pass at three
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

}  // namespace

bool train_radius_kernel(int block, int rh) { return forward_radius_kernel(block, rh); }

bool backward_radius_kernel(int block, int rh, int kc)
{
    return forward_radius_kernel(block, rh) && (kc == 24 || kc == 16 || kc == 8);
}

hipError_t launch_train_f32_radius(const StripArgs &a, hipStream_t s, int *occ)
{
    switch (a.rh) {
    case 3: return train_radius<3>(a, s, occ);
    case 5: return train_radius<5>(a, s, occ);
    case 8: return train_radius<8>(a, s, occ);
    case 10: return train_radius<10>(a, s, occ);
    case 16: return train_radius<16>(a, s, occ);
    case 20: return train_radius<20>(a, s, occ);
    case 25: return train_radius<25>(a, s, occ);
    case 32: return train_radius<32>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward_f32_radius(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    switch (a.rh) {
    case 3: return backward_radius<3>(a, kc, s, occ);
    case 5: return backward_radius<5>(a, kc, s, occ);
    case 8: return backward_radius<8>(a, kc, s, occ);
    case 10: return backward_radius<10>(a, kc, s, occ);
    case 16: return backward_radius<16>(a, kc, s, occ);
    case 20: return backward_radius<20>(a, kc, s, occ);
    case 25: return backward_radius<25>(a, kc, s, occ);
    case 32: return backward_radius<32>(a, kc, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bsk
