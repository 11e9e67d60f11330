// Single-image launches of the fused strip kernels (forward FP32/FP64 and
// precision forms, training forward, adjoint).  The kernel body and its
// design are in bsk_device.h, the strip kernel template in bsk_strip.h.
#include "bsk_strip.h"

namespace bsk {

// FP32 forward with the separable spatial kernel (NSC non-zero frequencies,
// SEVEN: the zero frequency present), one order per pipeline interval.
template <int BLOCK, int NSC, bool SEVEN>
constexpr int spatial_minb()
{
    return lds_occupancy(strip_lds_elems<PolForward<float>::NCH, 1, BLOCK, NSC, SEVEN>() * 4) >= 2 ? 2 : 1;
}
// RHC as for strip_kernel.
template <int BLOCK, int KR, int NSC, bool SEVEN, int RHC = 0>
__global__ void __launch_bounds__(BLOCK, (spatial_minb<BLOCK, NSC, SEVEN>())) spatial_kernel(const StripArgs a)
{
    __shared__ __align__(16) float lds[strip_lds_elems<PolForward<float>::NCH, 1, BLOCK, NSC, SEVEN>()];
    int bx, by;
    if (!xcd_tile(a.strips, (a.io.H + a.S - 1) / a.S, &bx, &by)) return;
    const Geom gm = geom_of(a);
    strip_body<float, BLOCK, KR, 1, PolForward<float>, 0, false, NSC, SEVEN, RHC>(a.io, gm, bx, by, lds, nullptr,
                                                                                  nullptr);
}

// Phase table of the spatial kernel: (cos, sin)(nu_j y) for y < n, the angle
// reduced modulo 2 pi in FP64 before rounding to FP32.
__global__ void __launch_bounds__(256) phase_table_kernel(int n, int nsc, double nu0, double nu1, double nu2,
                                                           float *tab)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * nsc) return;
    const int j = idx / n, y = idx - j * n;
    const double nu = j == 0 ? nu0 : j == 1 ? nu1 : nu2;
    double ang = nu * (double)y;
    ang -= 6.283185307179586 * rint(ang * 0.15915494309189535);
    tab[2 * idx] = (float)cos(ang);
    tab[2 * idx + 1] = (float)sin(ang);
}


// Fixed-order sum of the per-workgroup partials: grad_sigma = -(1/sigma) sum.
__global__ void __launch_bounds__(256) sigma_reduce_kernel(const float *unused, const double *part, int n,
                                                           double inv_sigma, float *out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) acc += part[q];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)(-inv_sigma * s[0]);
}

// ---------------------------------------------------------------- launches --
bool valid_chunk_forward_f32(int block, int kc)
{
    return kc == kr_f32(block) || kc == kr_f32(block) / 2;
}
bool valid_chunk_backward_f32(int block, int kc)
{
    return kc == kr_bwd(block) || kc == kr_bwd(block) / 2;
}
// A third pass size between the full and the half one, for 256-lane strips:
// 12 orders still fit three workgroups per CU (117 VGPRs for the plain FP32
// forward, 166 for the adjoint), and orders counts such as 22 then take two
// passes instead of three (or two padded ones of 16).
int mid_chunk_forward_f32(int block) { return block == 256 ? 12 : 0; }
// 20- and 24-order passes of the 256-lane plain FP32 forward at the
// compile-time radii still fit three workgroups per CU (150 and 166 VGPRs, no
// spill): many orders then take fewer passes, each of which repeats the
// recurrence starts of every row and the round trip of the partial
// accumulators through HBM.  (The run-time-radius R stage reads two prefixes
// per channel, and its one-pass 24-order kernel spills.)
int forward_chunks_f32(int block, int prec, int kahan, int rh, int *sizes)
{
    int n = 0;
    sizes[n++] = kr_f32(block);
    if (kr_f32(block) / 2 >= 1) sizes[n++] = kr_f32(block) / 2;
    if (block == 256 && prec == 0 && !kahan) {
        sizes[n++] = 12;
        if (forward_radius_kernel(block, rh)) {
            sizes[n++] = 20;
            sizes[n++] = 24;
        }
    }
    return n;
}
bool forward_chunk_ok_f32(int block, int prec, int kahan, int rh, int kc)
{
    int sizes[kMaxForwardChunks];
    const int n = forward_chunks_f32(block, prec, kahan, rh, sizes);
    for (int i = 0; i < n; ++i)
        if (sizes[i] == kc) return true;
    return false;
}
int mid_chunk_backward_f32(int block) { return block == 256 ? 12 : 0; }
// A 24-order adjoint pass for 256-lane strips (two workgroups per CU, 239
// VGPRs): 17 to 24 folded orders (N from 33 to 48) then take one pass instead
// of two padded ones of 16 (16 x 1024^2, N = 43: 1.67 -> 1.16 ms).
int big_chunk_backward_f32(int block) { return block == 256 ? 24 : 0; }
int chunk_forward_f32(int block) { return kr_f32(block); }
int chunk_forward_f64(int block) { return kr_f64(block); }
int chunk_train_f32(int block) { return kr_train(block); }
int chunk_backward_f32(int block) { return kr_bwd(block); }
int acc_count_forward() { return PolForward<float>::NACC; }
int acc_count_train() { return PolTrain<>::NACC; }
int acc_count_backward() { return PolBackward<>::NACC; }

template <int BLOCK, int QUANT, bool KAHAN>
static hipError_t fwd32_block(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    constexpr int KR = kr_f32(BLOCK), KL = kl_f32(BLOCK);
    // three workgroups per compute unit where the registers allow it
    constexpr int MINB = (BLOCK == 256 && !KAHAN) ? 3 : 0;
    if constexpr (BLOCK == 256 && QUANT == 0 && !KAHAN) {
        // the plain stack at a radius with its own kernels
        if ((kc == KR || kc == KR / 2) && forward_radius_kernel(BLOCK, a.rh))
            return launch_forward_f32_radius(a, kc, s, occ);
    }
    if constexpr (BLOCK == 256) {
        // one pass: the chain start mode as a constant (both pass sizes for the
        // plain FP32 stack, the full pass for the 16-bit and compensated ones)
        if (a.K <= kc && (a.start_mode == 0 || a.start_mode == 1)) {
            if (kc == KR)
                return a.start_mode == 0
                           ? launch<float, BLOCK, KR, KL, PolForward<float, 0>, QUANT, KAHAN, MINB>(a, s, occ)
                           : launch<float, BLOCK, KR, KL, PolForward<float, 1>, QUANT, KAHAN, MINB>(a, s, occ);
            if constexpr (QUANT == 0 && !KAHAN)
                return a.start_mode == 0
                           ? launch<float, BLOCK, KR / 2, KL, PolForward<float, 0>, 0, false, MINB>(a, s, occ)
                           : launch<float, BLOCK, KR / 2, KL, PolForward<float, 1>, 0, false, MINB>(a, s, occ);
        }
    }
    if (kc == KR) return launch<float, BLOCK, KR, KL, PolForward<float>, QUANT, KAHAN, MINB>(a, s, occ);
    return launch<float, BLOCK, KR / 2, KL, PolForward<float>, QUANT, KAHAN, MINB>(a, s, occ);
}

// The 12-order pass of the plain FP32 256-lane forward (one-pass launches with
// the start mode as a constant, like the other pass sizes).
static hipError_t fwd32_mid(const StripArgs &a, hipStream_t s, int *occ)
{
    constexpr int KR = 12, KL = 4;
    if (forward_radius_kernel(256, a.rh)) return launch_forward_f32_radius(a, KR, s, occ);
    if (a.K <= KR && (a.start_mode == 0 || a.start_mode == 1))
        return a.start_mode == 0 ? launch<float, 256, KR, KL, PolForward<float, 0>, 0, false, 3>(a, s, occ)
                                 : launch<float, 256, KR, KL, PolForward<float, 1>, 0, false, 3>(a, s, occ);
    return launch<float, 256, KR, KL, PolForward<float>, 0, false, 3>(a, s, occ);
}

template <int QUANT, bool KAHAN>
static hipError_t fwd32(const StripArgs &a, int block, int kc, hipStream_t s, int *occ)
{
    if constexpr (QUANT == 0 && !KAHAN) {
        if (block == 256 && kc == 12) return fwd32_mid(a, s, occ);
        // 20 and 24 orders: the compile-time radii only (forward_chunk_ok_f32)
        if (block == 256 && (kc == 20 || kc == 24)) return launch_forward_f32_radius(a, kc, s, occ);
    }
    switch (block) {
    case 256: return fwd32_block<256, QUANT, KAHAN>(a, kc, s, occ);
    case 512: return fwd32_block<512, QUANT, KAHAN>(a, kc, s, occ);
    case 1024: return fwd32_block<1024, QUANT, KAHAN>(a, kc, s, occ);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward_f32(const StripArgs &a, int block, int kc, int prec, int kahan, hipStream_t s, int *occ)
{
    if (!forward_chunk_ok_f32(block, prec, kahan, a.rh, kc)) return hipErrorInvalidValue;
    if (prec == 1) return kahan ? fwd32<1, true>(a, block, kc, s, occ) : fwd32<1, false>(a, block, kc, s, occ);
    if (prec == 2) return kahan ? fwd32<2, true>(a, block, kc, s, occ) : fwd32<2, false>(a, block, kc, s, occ);
    if (prec == 4) return kahan ? fwd32<4, true>(a, block, kc, s, occ) : fwd32<4, false>(a, block, kc, s, occ);
    return kahan ? fwd32<0, true>(a, block, kc, s, occ) : fwd32<0, false>(a, block, kc, s, occ);
}

// Two-pixel patch: the forward's shapes with the patch policy; the weights
// come from the device table of the call.
template <int BLOCK>
static hipError_t patch2_block(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    constexpr int KR = kr_f32(BLOCK), KL = kl_f32(BLOCK);
    constexpr int MINB = BLOCK == 256 ? 3 : 0;
    if (kc == KR) return launch<float, BLOCK, KR, KL, PolPatch2, 0, false, MINB>(a, s, occ);
    if (kc == KR / 2) return launch<float, BLOCK, KR / 2, KL, PolPatch2, 0, false, MINB>(a, s, occ);
    return hipErrorInvalidValue;
}

// Packed layout: the 256-lane full pass with groups of G orders, G = pack.
template <int G>
static hipError_t patch2_packed(const StripArgs &a, int pack, hipStream_t s, int *occ)
{
    if constexpr (G == 0) {
        return hipErrorInvalidValue;
    } else {
        constexpr int KR = kr_f32(256), KL = kl_f32(256);
        if (pack == G) return launch<float, 256, KR, KL, PolPatch2G<G>, 0, false, 3>(a, s, occ);
        return patch2_packed<G - 1>(a, pack, s, occ);
    }
}

hipError_t launch_patch2_f32(const StripArgs &a, int block, int kc, int pack, hipStream_t s, int *occ)
{
    static_assert(kr_f32(256) == kPatchPackPass, "packed patch kernels use the 256-lane full pass");
    if (pack != 0) {
        if (block != 256 || kc != kPatchPackPass || pack < 1 || pack > kPatchPackMax) return hipErrorInvalidValue;
        if (!occ && (!a.vf_dev || a.K % kc != 0)) return hipErrorInvalidValue;
        if (patch_radius_kernel(block, kc, a.rh)) return launch_patch2_f32_radius(a, pack, s, occ);
        return patch2_packed<kPatchPackMax>(a, pack, s, occ);
    }
    if (!occ && (!a.vf_dev || a.p2_group < kc || a.p2_group % kc != 0 || a.K % a.p2_group != 0))
        return hipErrorInvalidValue;
    if (patch_radius_kernel(block, kc, a.rh)) return launch_patch2_f32_radius(a, 0, s, occ);
    switch (block) {
    case 256: return patch2_block<256>(a, kc, s, occ);
    case 512: return patch2_block<512>(a, kc, s, occ);
    case 1024: return patch2_block<1024>(a, kc, s, occ);
    default: return hipErrorInvalidValue;
    }
}

// One-pass FP64 forward of 256 lanes: 16 orders in registers, two per
// interval (the three row buffers take 55 KiB, so two workgroups share a
// compute unit), with the chain start mode as a constant.  Up to 16 folded
// orders (N up to 31) then need no accumulator planes and one chain start
// per pixel and use.
constexpr int kr_f64_one(int block) { return block == 256 ? 16 : 0; }
int onepass_chunk_forward_f64(int block) { return kr_f64_one(block); }

hipError_t launch_forward_f64(const StripArgs &a, int block, int kc, hipStream_t s, int *occ)
{
    if (block == 256 && kc == kr_f64_one(256)) {
        constexpr int KR = kr_f64_one(256), KL = kl_f64(256);
        if (!occ && (a.K > KR || (a.start_mode != 0 && a.start_mode != 1))) return hipErrorInvalidValue;
        return a.start_mode == 1 ? launch<double, 256, KR, KL, PolForward<double, 1>, 0, false, 2>(a, s, occ)
                                 : launch<double, 256, KR, KL, PolForward<double, 0>, 0, false, 2>(a, s, occ);
    }
    if (kc != kr_f64(block)) return hipErrorInvalidValue;
    switch (block) {
    case 256: return launch<double, 256, kr_f64(256), kl_f64(256), PolForward<double>, 0, false>(a, s, occ);
    case 512: return launch<double, 512, kr_f64(512), kl_f64(512), PolForward<double>, 0, false>(a, s, occ);
    case 1024: return launch<double, 1024, kr_f64(1024), kl_f64(1024), PolForward<double>, 0, false>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_train_f32(const StripArgs &a, int block, int kc, hipStream_t s, int *occ)
{
    if (kc == kr_train(block) && train_radius_kernel(block, a.rh)) return launch_train_f32_radius(a, s, occ);
    // (a 12-order pass measured 6% slower than three of 8 on 22 orders at 1024^2,
    // and one 16-order pass at two workgroups per CU 3% slower than two of 8 on
    // 16 orders at 4096^2, and one 24-order pass 14% slower than three of 8 on 22
    // orders at 16 x 1024^2)
    if (kc != kr_train(block)) return hipErrorInvalidValue;
    switch (block) {
    case 256: return launch<float, 256, kr_train(256), kl_train(256), PolTrain<>, 0, false, 3>(a, s, occ);
    case 512: return launch<float, 512, kr_train(512), kl_train(512), PolTrain<>, 0, false>(a, s, occ);
    case 1024: return launch<float, 1024, kr_train(1024), kl_train(1024), PolTrain<>, 0, false>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}


template <int BLOCK>
static hipError_t bwd_block(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    constexpr int KR = kr_bwd(BLOCK), KL = kl_bwd(BLOCK);
    // a radius with its own kernels
    if (backward_radius_kernel(BLOCK, a.rh, kc)) return launch_backward_f32_radius(a, kc, s, occ);
    if constexpr (BLOCK == 256) {
        // one pass of 16 or 24 orders with the start mode as a constant (the
        // 16-order one then runs three workgroups per CU)
        if (a.K <= kc && (a.start_mode == 0 || a.start_mode == 1)) {
            if (kc == KR)
                return a.start_mode == 0 ? bwd<256, KR, KL, 0, 0, 0>(a, s, occ) : bwd<256, KR, KL, 0, 0, 1>(a, s, occ);
            if (kc == big_chunk_backward_f32(256))
                return a.start_mode == 0 ? bwd<256, 24, 4, 2, 0, 0>(a, s, occ) : bwd<256, 24, 4, 2, 0, 1>(a, s, occ);
        }
    }
    if (kc == KR) return bwd<BLOCK, KR, KL, 0>(a, s, occ);
    if constexpr (BLOCK == 256) {
        if (kc == mid_chunk_backward_f32(256)) return bwd<256, 12, 4, 3>(a, s, occ);
        if (kc == big_chunk_backward_f32(256)) return bwd<256, 24, 4, 2>(a, s, occ);
    }
    // the half pass of 256 lanes fits three workgroups per compute unit
    return bwd<BLOCK, KR / 2, (KL < KR / 2 ? KL : KR / 2), BLOCK == 256 ? 3 : 0>(a, s, occ);
}

// Spatial kernel: orders per pass by the number of frequencies (the complex
// running sums take 2 NSC registers per channel and order next to the plain
// one); a full pass and a small one (for few orders, e.g. Algorithm 1).
constexpr int kr_spatial(int nsc) { return nsc == 1 ? 4 : 2; }
constexpr int kr_spatial_small(int nsc) { return nsc == 1 ? 2 : 1; }
int chunk_spatial_f32(int block, int nsc)
{
    (void)block;
    return kr_spatial(nsc);
}
int chunk_spatial_small_f32(int block, int nsc)
{
    // the 512-lane strips offer the full pass only
    return block == 256 ? kr_spatial_small(nsc) : kr_spatial(nsc);
}
// 512-lane strips hold the LDS rows of at most two frequencies
bool spatial_block_ok(int block, int nsc) { return block == 256 || (block == 512 && nsc <= 2); }

template <int BLOCK, int NSC, bool SEVEN, int KR, int RHC = 0>
static hipError_t spatial_launch(const StripArgs &a, hipStream_t s, int *occ)
{
    if (occ) return query_occupancy((const void *)spatial_kernel<BLOCK, KR, NSC, SEVEN, RHC>, BLOCK, occ);
    if (RHC > 0 && a.rh != RHC) return hipErrorInvalidValue;
    const int Wt = BLOCK - 2 * a.rh;
    if (Wt < 1) return hipErrorInvalidValue;
    if (a.strips != (a.io.W + Wt - 1) / Wt) return hipErrorInvalidValue;
    const dim3 grid(xcd_grid(a.strips, strip_tiles(a) / a.strips));
    hipLaunchKernelGGL((spatial_kernel<BLOCK, KR, NSC, SEVEN, RHC>), grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// The q_2 kernel (one frequency and the constant term: three basis rows per
// channel, 16 walkers per row) has compile-time-radius kernels for the radii
// of the plain forward's, whose walkers hand out box sums.
template <int NSC, bool SEVEN, int KR>
static hipError_t spatial_radius(const StripArgs &a, hipStream_t s, int *occ)
{
    switch (a.rh) {
    case 3: return spatial_launch<256, NSC, SEVEN, KR, 3>(a, s, occ);
    case 5: return spatial_launch<256, NSC, SEVEN, KR, 5>(a, s, occ);
    case 8: return spatial_launch<256, NSC, SEVEN, KR, 8>(a, s, occ);
    case 10: return spatial_launch<256, NSC, SEVEN, KR, 10>(a, s, occ);
    case 16: return spatial_launch<256, NSC, SEVEN, KR, 16>(a, s, occ);
    case 20: return spatial_launch<256, NSC, SEVEN, KR, 20>(a, s, occ);
    case 25: return spatial_launch<256, NSC, SEVEN, KR, 25>(a, s, occ);
    case 32: return spatial_launch<256, NSC, SEVEN, KR, 32>(a, s, occ);
    default: return spatial_launch<256, NSC, SEVEN, KR>(a, s, occ);
    }
}

template <int BLOCK, int NSC, bool SEVEN>
static hipError_t spatial_go(const StripArgs &a, int kc, hipStream_t s, int *occ)
{
    if constexpr (BLOCK == 256 && NSC == 1 && SEVEN) {
        if (kc == kr_spatial(NSC)) return spatial_radius<NSC, SEVEN, kr_spatial(NSC)>(a, s, occ);
        if (kc == kr_spatial_small(NSC)) return spatial_radius<NSC, SEVEN, kr_spatial_small(NSC)>(a, s, occ);
    }
    if (kc == kr_spatial(NSC)) return spatial_launch<BLOCK, NSC, SEVEN, kr_spatial(NSC)>(a, s, occ);
    if constexpr (BLOCK == 256) {
        if (kc == kr_spatial_small(NSC)) return spatial_launch<BLOCK, NSC, SEVEN, kr_spatial_small(NSC)>(a, s, occ);
    }
    return hipErrorInvalidValue;
}

template <int BLOCK, int MAXNSC>
static hipError_t spatial_block(const StripArgs &a, const SpatialPlan &sp, int kc, hipStream_t s, int *occ)
{
    switch (sp.nsc * 2 + (sp.even ? 1 : 0)) {
    case 2: return spatial_go<BLOCK, 1, false>(a, kc, s, occ);
    case 3: return spatial_go<BLOCK, 1, true>(a, kc, s, occ);
    case 4: return spatial_go<BLOCK, 2, false>(a, kc, s, occ);
    case 5: return spatial_go<BLOCK, 2, true>(a, kc, s, occ);
    case 6:
        if constexpr (MAXNSC >= 3) return spatial_go<BLOCK, 3, false>(a, kc, s, occ);
        return hipErrorInvalidValue;
    case 7:
        if constexpr (MAXNSC >= 3) return spatial_go<BLOCK, 3, true>(a, kc, s, occ);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spatial_f32(const StripArgs &a, int block, const SpatialPlan &sp, int kc, hipStream_t s,
                              int *occ)
{
    if (!spatial_block_ok(block, sp.nsc)) return hipErrorInvalidValue;
    switch (block) {
    case 256: return spatial_block<256, 3>(a, sp, kc, s, occ);
    case 512: return spatial_block<512, 2>(a, sp, kc, s, occ);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_phase_table(const SpatialPlan &sp, int n, float *tab, hipStream_t s)
{
    const long total = (long)n * sp.nsc;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(phase_table_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, sp.nsc,
                       sp.nu[0], sp.nu[1], sp.nu[2], tab);
    return hipGetLastError();
}

hipError_t launch_backward_f32(const StripArgs &a, int block, int kc, float *grad_sigma, double inv_sigma,
                               int nred, hipStream_t s, int *occ)
{
    if (!valid_chunk_backward_f32(block, kc) && kc != mid_chunk_backward_f32(block) &&
        kc != big_chunk_backward_f32(block))
        return hipErrorInvalidValue;
    hipError_t e;
    switch (block) {
    case 256: e = bwd_block<256>(a, kc, s, occ); break;
    case 512: e = bwd_block<512>(a, kc, s, occ); break;
    case 1024: e = bwd_block<1024>(a, kc, s, occ); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || occ) return e;
    if (grad_sigma) {
        hipLaunchKernelGGL(sigma_reduce_kernel, dim3(1), dim3(256), 0, s, nullptr, (const double *)a.red, nred,
                           inv_sigma, grad_sigma);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace bsk
