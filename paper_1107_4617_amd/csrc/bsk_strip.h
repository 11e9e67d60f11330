// The strip kernels (single image, image stacks, adjoint) and their launch
// helpers, shared by the launch files (bsk_kernels.hip, bsk_poly.hip and the
// compile-time-radius files, bsk_radius.h).  The kernel body and its design
// are in bsk_device.h.
#pragma once
#include "bsk_device.h"

namespace bsk {

// Workgroups per compute unit that the LDS row buffers allow (160 KiB per CU,
// counted in 2 KiB units as in query_occupancy).
constexpr int lds_occupancy(int bytes) { return bytes <= 52 * 1024 ? 3 : bytes <= 80 * 1024 ? 2 : 1; }

// Pass shapes per lane count: KR orders in registers per pass and KL orders per
// pipeline interval (NCH * KL LDS rows per buffer).  The three row buffers stay
// under 54 KiB where the lane count allows it, so three 256-lane workgroups
// share a compute unit.  The half pass keeps KR / 2 orders in registers.
constexpr int kr_f32(int block) { return block == 256 ? 16 : block == 512 ? 8 : 4; }
constexpr int kl_f32(int block) { return block == 256 ? 4 : block == 512 ? 2 : 1; }
constexpr int kr_f64(int block) { return block == 256 ? 8 : block == 512 ? 4 : 1; }
constexpr int kl_f64(int block) { return block == 256 ? 2 : 1; }
// The adjoint offers a full and a half pass like the forward (the half pass
// of 256 lanes keeps three workgroups per CU).  The training forward box-sums
// six channels; eight orders per pass keep three 256-lane workgroups per CU.
constexpr int kr_bwd(int block) { return block == 256 ? 16 : block == 512 ? 8 : 2; }
constexpr int kl_bwd(int block) { return block == 256 ? 4 : block == 512 ? 2 : 1; }
constexpr int kr_train(int block) { return block == 256 ? 8 : block == 512 ? 6 : 2; }
constexpr int kl_train(int block) { return block == 1024 ? 1 : 2; }
template <int NCH, int KL, int BLOCK, typename AT>
constexpr int lds_elems() { return strip_lds_elems<NCH, KL, BLOCK>(); }
// workgroups per compute unit for the register allocation: what the LDS
// allows, at most two (three only where asked for explicitly)
template <int NCH, int KL, int BLOCK, typename AT>
constexpr int default_minb()
{
    return lds_occupancy(lds_elems<NCH, KL, BLOCK, AT>() * (int)sizeof(AT)) >= 2 ? 2 : 1;
}

// MINB: workgroups per compute unit the register allocation targets (0: the
// LDS-derived default).
__device__ __forceinline__ Geom geom_of(const StripArgs &a)
{
    Geom gm;
    gm.H = a.io.H;
    gm.W = a.io.W;
    gm.pitch_in = a.io.pitch_in;
    gm.pitch_out = a.io.pitch_out;
    gm.rh = a.rh;
    gm.rv = a.rv;
    gm.S = a.S;
    gm.K = a.K;
    gm.start_mode = a.start_mode;
    gm.omega_base = a.omega_base;
    gm.delta = a.delta;
    gm.v = a.v;
    gm.vf = a.vf;
    gm.ws = a.ws;
    gm.sp_u0 = a.sp_u0;
    for (int j = 0; j < kMaxSpatialFreq; ++j) gm.sp_u[j] = a.sp_u[j];
    gm.sp_row = a.sp_row;
    gm.sp_col = a.sp_col;
    gm.p2_group = a.p2_group;
    gm.p2_vf = a.vf_dev;
    gm.p2_omega1_base = a.p2_omega1_base;
    gm.p2_delta1 = a.p2_delta1;
    return gm;
}

// Tile of the launch's grid over a stack of images: its strip bx, the image b
// it lies in and its segment by within that image.  Returns false for the
// workgroups past the last tile.
__device__ __forceinline__ bool stack_tile(const StripArgs &a, int *bx, int *by, int *b)
{
    const int segs = (a.io.H + a.S - 1) / a.S;
    const int nimg = a.nimg > 1 ? a.nimg : 1;
    if (!xcd_tile(a.strips, segs * nimg, bx, by)) return false;
    *b = *by / segs;
    *by -= *b * segs;
    return true;
}
// Image b's buffers (a null buffer has a zero stride and stays null).
template <typename P>
__device__ __forceinline__ P at_image(P p, int b, long long bs)
{
    return (P)((const char *)p + b * bs);
}
__device__ __forceinline__ IO stack_io(const StripArgs &a, int b)
{
    IO io = a.io;
    io.img = at_image(io.img, b, a.bs_img);
    io.out = at_image(io.out, b, a.bs_out);
    io.out2 = at_image(io.out2, b, a.bs_out2);
    io.aux0 = at_image(io.aux0, b, a.bs_aux[0]);
    io.aux1 = at_image(io.aux1, b, a.bs_aux[1]);
    io.aux2 = at_image(io.aux2, b, a.bs_aux[2]);
    io.aux3 = at_image(io.aux3, b, a.bs_aux[3]);
    io.aux4 = at_image(io.aux4, b, a.bs_aux[4]);
    return io;
}
__device__ __forceinline__ Geom stack_geom(const StripArgs &a, int b)
{
    Geom gm = geom_of(a);
    gm.ws = at_image(gm.ws, b, a.bs_ws);
    return gm;
}

// RHC > 0: the horizontal window radius as a compile-time constant (the
// launch's rh must equal it); 0: the run-time radius.
template <typename AT, int BLOCK, int KR, int KL, class POL, int QUANT, bool KAHAN, int MINB = 0, int RHC = 0>
__global__ void __launch_bounds__(BLOCK, MINB ? MINB : (default_minb<POL::NCH, KL, BLOCK, AT>()))
    strip_kernel(const StripArgs a)
{
    __shared__ __align__(16) AT lds[lds_elems<POL::NCH, KL, BLOCK, AT>()];
    int bx, by;
    if constexpr (std::is_same<POL, PolTrain<POL::START>>::value) {
        // the training forward also runs over image stacks
        int b;
        if (!stack_tile(a, &bx, &by, &b)) return;
        const IO io = stack_io(a, b);
        const Geom gm = stack_geom(a, b);
        strip_body<AT, BLOCK, KR, KL, POL, QUANT, KAHAN, 0, true, RHC>(io, gm, bx, by, lds, nullptr, nullptr);
    } else {
        if (!xcd_tile(a.strips, (a.io.H + a.S - 1) / a.S, &bx, &by)) return;
        const Geom gm = geom_of(a);
        strip_body<AT, BLOCK, KR, KL, POL, QUANT, KAHAN, 0, true, RHC>(a.io, gm, bx, by, lds, nullptr, nullptr);
    }
}

// The adjoint over a stack of images; RHC as for strip_kernel, SM >= 0 a
// one-pass launch (K <= KR) with that chain start mode.
template <int BLOCK, int KR, int KL, int MINB = 0, int RHC = 0, int SM = -1>
__global__ void __launch_bounds__(BLOCK, MINB ? MINB : (default_minb<PolBackward<>::NCH, KL, BLOCK, float>()))
    backward_kernel(const StripArgs a)
{
    // the block reduction of the sigma_r partial sums reuses the row buffers
    // once the rows are done, so it adds no LDS (three workgroups per compute
    // unit fit where the row buffers alone allow it)
    constexpr int NL = lds_elems<PolBackward<>::NCH, KL, BLOCK, float>();
    static_assert(NL * sizeof(float) >= BLOCK * sizeof(double), "the reduction fits in the row buffers");
    __shared__ __align__(16) float lds[NL];
    double *const red_lds = reinterpret_cast<double *>(lds);
    int bx, by, b;
    if (!stack_tile(a, &bx, &by, &b)) return;
    const IO io = stack_io(a, b);
    const Geom gm = stack_geom(a, b);
    // one partial sum per tile of the whole stack, image-major like the tiles
    const long segs = (a.io.H + a.S - 1) / a.S;
    strip_body<float, BLOCK, KR, KL, PolBackward<SM>, 0, false, 0, true, RHC>(
        io, gm, bx, by, lds, red_lds, a.red + (((long)b * segs + by) * a.strips + bx));
}

// ---------------------------------------------------------------- launches --
// Every launch helper either launches (occ == nullptr) or reports, in *occ,
// how many workgroups of that exact kernel one compute unit holds.
// The runtime's answer is capped by the kernel's LDS counted in 2 KiB units
// out of 160 KiB: a 53 KiB workgroup (54,272 bytes) that the runtime placed
// three to a compute unit ran only two at a time, which sized a launch for one
// and a half rounds of workgroups; 51 KiB ones do run three at a time.
inline hipError_t query_occupancy(const void *kernel, int block, int *occ)
{
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0);
    *occ = (e == hipSuccess && n > 0) ? n : 1;
    hipFuncAttributes fa;
    if (e == hipSuccess && hipFuncGetAttributes(&fa, kernel) == hipSuccess && fa.sharedSizeBytes > 0) {
        constexpr long kUnit = 2048, kLds = 160 * 1024;
        const long units = ((long)fa.sharedSizeBytes + kUnit - 1) / kUnit;
        const int by_lds = (int)(kLds / (units * kUnit));
        if (by_lds >= 1 && *occ > by_lds) *occ = by_lds;
    }
    return e;
}

template <typename AT, int BLOCK, int KR, int KL, class POL, int QUANT, bool KAHAN, int MINB = 0, int RHC = 0>
static hipError_t launch(const StripArgs &a, hipStream_t s, int *occ)
{
    if (occ)
        return query_occupancy((const void *)strip_kernel<AT, BLOCK, KR, KL, POL, QUANT, KAHAN, MINB, RHC>, BLOCK, occ);
    if (RHC > 0 && a.rh != RHC) return hipErrorInvalidValue;
    if (POL::START >= 0 && (a.K > KR || a.start_mode != POL::START)) return hipErrorInvalidValue;
    const int Wt = BLOCK - 2 * a.rh;
    if (Wt < 1) return hipErrorInvalidValue;
    if (a.strips != (a.io.W + Wt - 1) / Wt) return hipErrorInvalidValue;
    const dim3 grid(xcd_grid(a.strips, strip_tiles(a) / a.strips));
    hipLaunchKernelGGL((strip_kernel<AT, BLOCK, KR, KL, POL, QUANT, KAHAN, MINB, RHC>), grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int BLOCK, int KR, int KL, int MINB, int RHC = 0, int SM = -1>
static hipError_t bwd(const StripArgs &a, hipStream_t s, int *occ)
{
    if (occ) return query_occupancy((const void *)backward_kernel<BLOCK, KR, KL, MINB, RHC, SM>, BLOCK, occ);
    if (RHC > 0 && a.rh != RHC) return hipErrorInvalidValue;
    if (SM >= 0 && (a.K > KR || a.start_mode != SM)) return hipErrorInvalidValue;
    const int Wt = BLOCK - 2 * a.rh;
    if (Wt < 1) return hipErrorInvalidValue;
    if (a.strips != (a.io.W + Wt - 1) / Wt) return hipErrorInvalidValue;
    const dim3 grid(xcd_grid(a.strips, strip_tiles(a) / a.strips));
    hipLaunchKernelGGL((backward_kernel<BLOCK, KR, KL, MINB, RHC, SM>), grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace bsk
