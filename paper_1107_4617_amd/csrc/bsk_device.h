// Device code shared by the strip kernels of the constant-time bilateral filter (gfx950).
//
// Algorithm 2 of the paper with one spatial basis function (the box) and the
// folded raised-cosine range kernel computes, for every pixel x,
//     Q(x) = sum_m v_m [C_m(x) Box[C_m](x) + S_m(x) Box[S_m](x)]
//     P(x) = sum_m v_m [C_m(x) Box[f C_m](x) + S_m(x) Box[f S_m](x)]
//     out(x) = P(x) / Q(x)
// with C_m = cos(omega_m f), S_m = sin(omega_m f) (step 1, the pointwise
// transforms), Box = the moving sum Sum(F, x, r) of Section 2 (step 2) and the
// shift identity cos(a - b) = cos a cos b + sin a sin b to recombine (step 3).
//
// Mapping onto the GPU.  A workgroup owns a strip of BLOCK image columns (its
// Wt = BLOCK - 2 rh output columns plus rh halo columns on each side) and a
// segment of S output rows, which it walks from top to bottom.  Lane t owns
// column j0 - rh + t.  Per output row i, for each group of KL orders:
//   stage V  every lane updates, in registers, the vertical moving sums of all
//            channels of its column: V += X(i + rv) - X(i - rv - 1).  The
//            transforms X come from a three-term recurrence over the orders
//            (one sincos per pixel), so cos/sin are never evaluated per order.
//            V is written to an LDS row buffer.
//   stage H  "walker" lanes turn each LDS row into its exclusive prefix sums
//            E in place: each walker scans a chunk of the row in registers and
//            the chunk totals are combined by a scan across the row's walkers.
//   stage R  every output lane forms the horizontal box sums as prefix
//            differences B(j) = E(j + rh + 1) - E(j - rh) and recombines its
//            pixel from the box sums and the transforms of its own value.
// The three stages are software-pipelined over three row buffers (see
// strip_body).  The (channels x orders) stack therefore lives only in
// registers and LDS; HBM sees the input (read ~3 times through L2: as
// incoming, centre and outgoing row, each load issued one row ahead) and the
// output.  Values are centred on a per-workgroup reference level before
// transforming (the filter is shift covariant), which halves the magnitude of
// the f-weighted sums.  The order count is padded to a multiple of the pass
// size with zero weights, so every pass runs the same straight-line code;
// passes after the first continue from partial accumulators kept in a
// workspace.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <type_traits>

#include "bsk_internal.h"

namespace bsk {

// ------------------------------------------------------------------ helpers --
// sin and cos of a float angle: Cody-Waite reduction by pi/2 done in FP64
// (exact enough for |x| up to ~1e6), then the Taylor polynomials of sin and cos
// on [-pi/4, pi/4] (truncation error below 2e-9), and the quadrant rotation.
// Branch-free, about twenty VALU instructions.
__device__ __forceinline__ void poly_sincos(float x, float *s, float *c)
{
    const float k = rintf(x * 0.636619772367581343f);   // 2/pi
    const float r = (float)__builtin_fma(-(double)k, 1.5707963267948966, (double)x);
    const float r2 = r * r;
    float ps = __builtin_fmaf(r2, 2.75573192239858907e-6f, -1.98412698412698413e-4f);
    ps = __builtin_fmaf(r2, ps, 8.33333333333333333e-3f);
    ps = __builtin_fmaf(r2, ps, -1.66666666666666667e-1f);
    const float sr = __builtin_fmaf(r * r2, ps, r);
    float pc = __builtin_fmaf(r2, -2.75573192239858907e-7f, 2.48015873015873016e-5f);
    pc = __builtin_fmaf(r2, pc, -1.38888888888888889e-3f);
    pc = __builtin_fmaf(r2, pc, 4.16666666666666667e-2f);
    pc = __builtin_fmaf(r2, pc, -0.5f);
    const float cr = __builtin_fmaf(r2, pc, 1.0f);
    const int q = (int)k;
    const float sv = (q & 1) ? cr : sr;
    const float cv = (q & 1) ? sr : cr;
    *s = (q & 2) ? -sv : sv;
    *c = ((q + 1) & 2) ? -cv : cv;
}
// sin and cos of a float angle on the transcendental unit (v_sin_f32 /
// v_cos_f32 take the angle in revolutions and reduce it themselves): one
// product and two instructions.  Angles beyond +-1600 radians (the unit's
// +-256 revolutions) take the polynomial path.  The recurrence starts use it;
// the GPU parity tests hold the filter to the same error as the polynomials
// (headline: max 5.9e-4 against the FP64 oracle, 4.6e-4 with the polynomials).
__device__ __forceinline__ void fast_sincos(float x, float *s, float *c)
{
    if (fabsf(x) > 1600.0f) {
        poly_sincos(x, s, c);
        return;
    }
    const float rev = x * 0.159154943091895336f;   // 1 / (2 pi)
    *s = __builtin_amdgcn_sinf(rev);
    *c = __builtin_amdgcn_cosf(rev);
}
__device__ __forceinline__ void sc(float x, float *s, float *c) { fast_sincos(x, s, c); }

// sin and cos of y for |y| <= pi/2 (the half step angle of the recurrence):
// the transcendental unit, as fast_sincos.
__device__ __forceinline__ void sincos_small(float y, float *s, float *c) { fast_sincos(y, s, c); }
__device__ __forceinline__ void sc_small(float y, float *s, float *c) { sincos_small(y, s, c); }
// FP64: the Taylor polynomials to degree 21 and 22 (truncation error below
// 2e-18 at |y| = pi/2), no reduction; the library's sincos beyond pi/2.
__device__ __forceinline__ void sc_small(double y, double *s, double *c)
{
    if (fabs(y) > 1.5707963267948966) {
        sincos(y, s, c);
        return;
    }
    const double y2 = y * y;
    // coefficients (-1)^k / (2k+1)! and (-1)^k / (2k)!
    double ps = __builtin_fma(y2, -1.9572941063391263e-20, 8.2206352466243297e-18);
    ps = __builtin_fma(y2, ps, -2.8114572543455208e-15);
    ps = __builtin_fma(y2, ps, 7.6471637318198164e-13);
    ps = __builtin_fma(y2, ps, -1.6059043836821613e-10);
    ps = __builtin_fma(y2, ps, 2.5052108385441720e-08);
    ps = __builtin_fma(y2, ps, -2.7557319223985893e-06);
    ps = __builtin_fma(y2, ps, 1.9841269841269841e-04);
    ps = __builtin_fma(y2, ps, -8.3333333333333332e-03);
    ps = __builtin_fma(y2, ps, 1.6666666666666666e-01);
    *s = __builtin_fma(-y * y2, ps, y);
    double pc = __builtin_fma(y2, 8.8967913924505741e-22, -4.1103176233121649e-19);
    pc = __builtin_fma(y2, pc, 1.5619206968586225e-16);
    pc = __builtin_fma(y2, pc, -4.7794773323873853e-14);
    pc = __builtin_fma(y2, pc, 1.1470745597729725e-11);
    pc = __builtin_fma(y2, pc, -2.0876756987868099e-09);
    pc = __builtin_fma(y2, pc, 2.7557319223985888e-07);
    pc = __builtin_fma(y2, pc, -2.4801587301587302e-05);
    pc = __builtin_fma(y2, pc, 1.3888888888888889e-03);
    pc = __builtin_fma(y2, pc, -4.1666666666666664e-02);
    pc = __builtin_fma(y2, pc, 0.5);
    *c = __builtin_fma(-y2, pc, 1.0);
}
// reciprocal: the hardware approximation in FP32 (about 1 ulp), a divide in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
// fused multiply-add in the type of its arguments
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ void sc(double x, double *s, double *c) { sincos(x, s, c); }

// sin and cos of a recurrence step d = delta g: the half angle by the
// polynomials without reduction (|d| <= pi when the order is at least N_0 and
// the data span at most T; beyond that sc_small reduces), then the double-angle
// formulas.
template <typename AT>
__device__ __forceinline__ void sc_step(AT d, AT *s, AT *c)
{
    AT sh, ch;
    sc_small(AT(0.5) * d, &sh, &ch);
    *c = fmat(AT(-2) * sh, sh, AT(1));
    *s = AT(2) * sh * ch;
}

// Stack quantisation of the precision forms: 1 bfloat16, 2 float16 (both round
// to nearest even), 4 signed 16-bit fixed point with 15 fraction bits (the
// basis values lie in [-1, 1]); 0 leaves FP32 values untouched.
template <int QUANT>
__device__ __forceinline__ float quant(float x)
{
    if constexpr (QUANT == 1) return __bfloat162float(__float2bfloat16(x));
    else if constexpr (QUANT == 2) return __half2float(__float2half_rn(x));
    else if constexpr (QUANT == 4) return rintf(x * 32767.0f) * (1.0f / 32767.0f);
    else return x;
}
template <int QUANT>
__device__ __forceinline__ double quant(double x) { return x; }

// cos and sin of (omega_0 + m delta) g for m = 0, 1, ... by the three-term
// recurrence x_{m+1} = 2 cos(delta g) x_m - x_{m-1}, which both sequences
// satisfy (angle addition); one fused multiply-add per value and order.  The
// start needs one sincos of the half step angle when omega_0 is 0 or delta / 2
// (the first pass of an even or odd order), two general sincos otherwise.  A
// pixel outside the image starts at zero so all its channels vanish.
template <typename AT>
struct Chain {
    AT c, s, cp, sp, a2;   // current, previous, 2 cos(delta g)
    // M >= 0: the start mode is that compile-time constant (one-pass launches);
    // M < 0: the run-time `mode`, resolved with selects (a branch per mode
    // measured slower there).
    template <int M = -1>
    __device__ __forceinline__ void start(bool valid, AT g, AT om0, AT dlt, int mode)
    {
        if constexpr (M == 0 || M == 1) {
            // the half step angle y = delta g / 2, then the step by the double-angle formulas
            AT sh, ch;
            sc_small(AT(0.5) * dlt * g, &sh, &ch);
            const AT cd = fmat(AT(-2) * sh, sh, AT(1));
            a2 = AT(2) * cd;
            if constexpr (M == 0) {
                // omega_0 = 0: (c, s) = (1, 0) and the order before it at -delta g
                const AT sd = AT(2) * sh * ch;
                c = valid ? AT(1) : AT(0);
                s = AT(0);
                cp = valid ? cd : AT(0);
                sp = valid ? -sd : AT(0);
            } else {
                // omega_0 = delta / 2 = y / g: (c, s) = (ch, sh) and the order before it at -y
                c = valid ? ch : AT(0);
                s = valid ? sh : AT(0);
                cp = c;
                sp = -s;
            }
        } else {
            AT c0, s0, cd, sd;
            if (mode <= 1) {
                // the half step angle y = delta g / 2 (= omega_0 g when omega_0 = delta / 2),
                // then the step by the double-angle formulas
                AT sh, ch;
                sc_small(AT(0.5) * dlt * g, &sh, &ch);
                cd = fmat(AT(-2) * sh, sh, AT(1));
                sd = AT(2) * sh * ch;
                c0 = mode == 0 ? AT(1) : ch;
                s0 = mode == 0 ? AT(0) : sh;
            } else {
                sc(om0 * g, &s0, &c0);
                sc_step(dlt * g, &sd, &cd);
            }
            const AT z = valid ? AT(1) : AT(0);
            c = z * c0;
            s = z * s0;
            cp = z * (c0 * cd + s0 * sd);   // (cos, sin) of (omega_0 - delta) g
            sp = z * (s0 * cd - c0 * sd);
            a2 = AT(2) * cd;
        }
    }
    // S0: the current sine value is exactly zero (the zero frequency), so the
    // next one is -sp without a multiply-add on the zero
    template <bool S0 = false>
    __device__ __forceinline__ void step()
    {
        const AT cn = fmat(a2, c, -cp);
        const AT sn = S0 ? -sp : fmat(a2, s, -sp);
        cp = c;
        sp = s;
        c = cn;
        s = sn;
    }
};

// The chain of a two-pixel-patch pass: phases omega_1 g_1 + (omega_0 + m delta) g_2
// of one first-pixel frequency omega_1.  A pass may hold several first-pixel
// frequencies, omega_1 + j delta_1, each with the same run of second-pixel
// orders; the chain then restarts at the next frequency's first order by
// rotating that frequency's starting phase by delta_1 g_1 (one complex
// multiplication), with no further sincos.
template <typename AT>
struct PatchChain : Chain<AT> {
    AT gc, gs;     // (cos, sin) of the current frequency's starting phase
    AT r1c, r1s;   // (cos, sin)(delta_1 g_1)
    AT sd;         // sin(delta g_2)
    // start at phase psi with steps d2 = delta g_2 (orders) and d1 = delta_1 g_1
    // (first-pixel frequencies)
    __device__ __forceinline__ void start_patch(bool valid, AT psi, AT d2, AT d1)
    {
        AT c0, s0, cd;
        sc(psi, &s0, &c0);
        sc_step(d2, &sd, &cd);
        sc_step(d1, &r1s, &r1c);
        const AT z = valid ? AT(1) : AT(0);
        this->c = gc = z * c0;
        this->s = gs = z * s0;
        this->cp = z * (c0 * cd + s0 * sd);
        this->sp = z * (s0 * cd - c0 * sd);
        this->a2 = AT(2) * cd;
    }
    __device__ __forceinline__ void restart()
    {
        const AT nc = fmat(gc, r1c, -gs * r1s);
        const AT ns = fmat(gs, r1c, gc * r1s);
        gc = nc;
        gs = ns;
        const AT cd = AT(0.5) * this->a2;
        this->c = nc;
        this->s = ns;
        this->cp = fmat(nc, cd, ns * sd);
        this->sp = fmat(ns, cd, -nc * sd);
    }
};

template <typename T>
__device__ __forceinline__ T ld(const void *p, long idx) { return ((const T *)p)[idx]; }

// ------------------------------------------------------------------ policies --
// A policy fixes the channels that are box-summed per order, the raw per-pixel
// inputs they need (fetched one row ahead), and how box sums recombine into
// per-pixel accumulators.  fetch always reads the in-image pixel (i, j) it is
// given (callers clamp the indices) and replaces it by the value of an absent
// pixel when valid is false, so that loads never need a branch.

// Channels come in pairs (kappa_p C, kappa_p S) with a per-pixel coefficient
// kappa_p; channel 2p is the cosine member and 2p+1 the sine member.

// Forward: channels (C, S, gC, gS), g = f - ref; accumulators (Q, P).  SM >= 0
// fixes a one-pass launch (K <= KR) whose chain start mode is SM (0: even N,
// 1: odd N), so the start's selects and the general-angle path compile away.
template <typename FT, int SM = -1>
struct PolForward {
    static constexpr int NCH = 4, NACC = 2, NAUX = 1, NRAW = 1, NPAIR = 2, NCTR = 0;
    static constexpr int START = SM;
    template <typename AT>
    __device__ static void kappa(const AT *aux, AT *k)
    {
        k[0] = AT(1);
        k[1] = aux[0];
    }
    template <typename AT>
    __device__ static AT ref(const IO &a, int i, int j)
    {
        return (AT)ld<FT>(a.img, (long)i * a.pitch_in + j);
    }
    template <typename AT>
    __device__ static void fetch(const IO &a, bool valid, int i, int j, AT *raw)
    {
        const AT x = (AT)ld<FT>(a.img, (long)i * a.pitch_in + j);
        raw[0] = valid ? x : AT(0);
    }
    template <typename AT>
    __device__ static void make(const AT *raw, AT ref, AT *aux)
    {
        aux[0] = raw[0] - ref;
    }
    template <typename AT>
    __device__ static void chans(AT C, AT S, const AT *aux, AT *X)
    {
        X[0] = C;
        X[1] = S;
        X[2] = aux[0] * C;
        X[3] = aux[0] * S;
    }
    // accumulated as two chained multiply-adds per accumulator
    template <typename AT>
    __device__ static void recombine(AT v, AT vom, AT C, AT S, const AT *B, const AT *auxc, AT *acc)
    {
        const AT vc = v * C, vs = v * S;
        acc[0] = fmat(vc, B[0], fmat(vs, B[1], acc[0]));
        acc[1] = fmat(vc, B[2], fmat(vs, B[3], acc[1]));
    }
    // the zero frequency: S = 0, so only the cosine members contribute
    template <typename AT>
    __device__ static void recombine_s0(AT v, AT C, const AT *B, AT *acc)
    {
        const AT vc = v * C;
        acc[0] = fmat(vc, B[0], acc[0]);
        acc[1] = fmat(vc, B[2], acc[1]);
    }
    template <typename AT>
    __device__ static void finalize(const IO &a, int i, int j, AT ref, const AT *auxc, const AT *acc,
                                    const AT *ctr, double *red)
    {
        ((FT *)a.out)[(long)i * a.pitch_out + j] = (FT)(ref + acc[1] / acc[0]);
    }
};

// Two-pixel-patch non-local means (Section 5 with p = 2): the range kernel
// compares the patches {z, z + u} through cos^N1(w t_1) cos^N2(w' t_2), whose
// expansion holds terms cos(omega_1 t_1 + omega_2 t_2).  A term's channels are
// those of the forward policy with the patch phase
// psi(z) = omega_1 g(z) + omega_2 g(z + u) in place of omega g(z); the second
// patch pixel lies beyond the image only through the clamped read (the image
// extended by its nearest border pixel).
// G > 0 packs KR / G first-pixel frequencies of G orders each into every pass
// (their chains restart at orders G, 2G, ..); G = 0 runs one frequency's
// orders per pass range.
template <int G>
struct PolPatch2G {
    static constexpr int NCH = 4, NACC = 2, NAUX = 2, NRAW = 2, NPAIR = 2, NCTR = 0;
    static constexpr int START = -1;
    static constexpr int GROUP = G;
    template <typename AT>
    __device__ static void kappa(const AT *aux, AT *k)
    {
        k[0] = AT(1);
        k[1] = aux[0];
    }
    template <typename AT>
    __device__ static AT ref(const IO &a, int i, int j)
    {
        return (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
    }
    template <typename AT>
    __device__ static void fetch(const IO &a, bool valid, int i, int j, AT *raw)
    {
        const int i2 = min(max(i + a.uy, 0), a.H - 1);
        const int j2 = min(max(j + a.ux, 0), a.W - 1);
        const AT x = (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
        const AT x2 = (AT)ld<float>(a.img, (long)i2 * a.pitch_in + j2);
        raw[0] = valid ? x : AT(0);
        raw[1] = valid ? x2 : AT(0);
    }
    template <typename AT>
    __device__ static void make(const AT *raw, AT ref, AT *aux)
    {
        aux[0] = raw[0] - ref;
        aux[1] = raw[1] - ref;
    }
    template <typename AT>
    __device__ static void recombine(AT v, AT vom, AT C, AT S, const AT *B, const AT *auxc, AT *acc)
    {
        PolForward<float>::recombine<AT>(v, vom, C, S, B, auxc, acc);
    }
    template <typename AT>
    __device__ static void finalize(const IO &a, int i, int j, AT ref, const AT *auxc, const AT *acc,
                                    const AT *ctr, double *red)
    {
        ((float *)a.out)[(long)i * a.pitch_out + j] = (float)(ref + acc[1] / acc[0]);
    }
};
template <class P>
struct IsPatch2 {
    static constexpr bool value = false;
};
template <int G>
struct IsPatch2<PolPatch2G<G>> {
    static constexpr bool value = true;
};
using PolPatch2 = PolPatch2G<0>;
template <class P>
struct IsForward32 {
    static constexpr bool value = false;
};
template <int SM>
struct IsForward32<PolForward<float, SM>> {
    static constexpr bool value = true;
};

// The chain type of a policy: the patch's restartable chain, else the plain one.
template <class POL, typename AT>
struct ChainOf {
    using type = Chain<AT>;
};
template <int G, typename AT>
struct ChainOf<PolPatch2G<G>, AT> {
    using type = typename std::conditional<(G > 0), PatchChain<AT>, Chain<AT>>::type;
};

// Start of an order chain: the angle omega g of one value, or for the
// two-pixel patch the phase omega_1 g_1 + omega_2 g_2 (om1 = omega_1) with the
// step delta g_2 of the second value and, when a pass holds several first-pixel
// frequencies, the rotation by delta_1 g_1 between them (d1 = delta_1).
template <class POL, typename AT, class CH>
__device__ __forceinline__ void chain_start(CH &ch, bool valid, const AT *aux, AT om0, AT dlt, int mode, AT om1,
                                            AT d1)
{
    if constexpr (IsPatch2<POL>::value) {
        if constexpr (POL::GROUP > 0)
            ch.start_patch(valid, fmat(om1, aux[0], om0 * aux[1]), dlt * aux[1], d1 * aux[0]);
        else
            ch.start(valid, AT(1), fmat(om1, aux[0], om0 * aux[1]), dlt * aux[1], 2);
    } else {
        ch.template start<POL::START>(valid, aux[0], om0, dlt, mode);
    }
}

// Before order m of a pass (m a constant of the unrolled loops): a packed patch
// chain moves on to the next first-pixel frequency at every multiple of G.
template <class POL, class CH>
__device__ __forceinline__ void chain_restart(CH &ch, int m)
{
    if constexpr (IsPatch2<POL>::value) {
        if constexpr (POL::GROUP > 0) {
            if (m > 0 && m % POL::GROUP == 0) ch.restart();
        }
    }
}

// Training forward: channels (C, S, gC, gS, g^2 C, g^2 S); accumulators
// (Q, P, A0, A1, A2) with A_p(z) = sum_{y in B(z)} phi'(g_y - g_z) g_y^p
//   = -sum_m v_m omega_m [C_m(z) Box[g^p S_m] - S_m(z) Box[g^p C_m]],
// phi'(t) = -sum_m v_m omega_m sin(omega_m t).  Outputs u = ref + P/Q and the
// planes Q, E1 = A1 - (u-ref) A0, E2 = A2 - (g_z + u - ref) A1 + g_z (u-ref) A0.
// SM >= 0 fixes a one-pass launch's chain start mode, as for the forward.
template <int SM = -1>
struct PolTrain {
    static constexpr int NCH = 6, NACC = 5, NAUX = 1, NRAW = 1, NPAIR = 3, NCTR = 0;
    static constexpr int START = SM;
    template <typename AT>
    __device__ static void kappa(const AT *aux, AT *k)
    {
        k[0] = AT(1);
        k[1] = aux[0];
        k[2] = aux[0] * aux[0];
    }
    template <typename AT>
    __device__ static AT ref(const IO &a, int i, int j)
    {
        return (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
    }
    template <typename AT>
    __device__ static void fetch(const IO &a, bool valid, int i, int j, AT *raw)
    {
        const AT x = (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
        raw[0] = valid ? x : AT(0);
    }
    template <typename AT>
    __device__ static void make(const AT *raw, AT ref, AT *aux)
    {
        aux[0] = raw[0] - ref;
    }
    template <typename AT>
    __device__ static void chans(AT C, AT S, const AT *aux, AT *X)
    {
        const AT g = aux[0];
        X[0] = C;
        X[1] = S;
        X[2] = g * C;
        X[3] = g * S;
        X[4] = g * X[2];
        X[5] = g * X[3];
    }
    template <typename AT>
    __device__ static void recombine(AT v, AT vom, AT C, AT S, const AT *B, const AT *auxc, AT *acc)
    {
        const AT vc = v * C, vs = v * S;
        acc[0] = fmat(vc, B[0], fmat(vs, B[1], acc[0]));
        acc[1] = fmat(vc, B[2], fmat(vs, B[3], acc[1]));
        const AT wc = vom * C, ws = vom * S;
        acc[2] = fmat(ws, B[0], fmat(-wc, B[1], acc[2]));
        acc[3] = fmat(ws, B[2], fmat(-wc, B[3], acc[3]));
        acc[4] = fmat(ws, B[4], fmat(-wc, B[5], acc[4]));
    }
    // the zero frequency: S = 0 and omega = 0, so the A_p terms vanish
    template <typename AT>
    __device__ static void recombine_s0(AT v, AT C, const AT *B, AT *acc)
    {
        const AT vc = v * C;
        acc[0] = fmat(vc, B[0], acc[0]);
        acc[1] = fmat(vc, B[2], acc[1]);
    }
    template <typename AT>
    __device__ static void finalize(const IO &a, int i, int j, AT ref, const AT *auxc, const AT *acc,
                                    const AT *ctr, double *red)
    {
        const AT Q = acc[0];
        const AT ut = acc[1] / Q;
        const AT gz = auxc[0];
        const long plane = (long)a.H * a.W;
        const long o = (long)i * a.W + j;
        ((float *)a.out)[(long)i * a.pitch_out + j] = (float)(ref + ut);
        a.out2[o] = (float)Q;
        a.out2[plane + o] = (float)(acc[3] - ut * acc[2]);
        a.out2[2 * plane + o] = (float)(acc[4] - (gz + ut) * acc[3] + gz * ut * acc[2]);
    }
};

// Policies whose recombination uses each order's weight only as a factor of
// all its box-sum terms (v_m, or v_m omega_m): the H stage then scales the
// prefix rows of order m by v_m, and the R stage takes v = 1 and omega_m in
// place of v_m omega_m.
template <class P>
struct FoldsWeight {
    static constexpr bool value = false;
};
template <typename FT, int SM>
struct FoldsWeight<PolForward<FT, SM>> {
    static constexpr bool value = true;
};
template <int SM>
struct FoldsWeight<PolTrain<SM>> {
    static constexpr bool value = true;
};
// the two-pixel patch's weight table (w1[g] v_m per packed order) scales the
// walker rows the same way
template <int G>
struct FoldsWeight<PolPatch2G<G>> {
    static constexpr bool value = true;
};

// Backward (adjoint): with alpha = gbar / Q and ut = u - ref, channels
// (alpha C, alpha S, alpha ut C, alpha ut S); one accumulator
//   T1(z) = sum_m v_m { C(z) Box[aC] + S(z) Box[aS]
//           - omega_m [ S(z) (g_z Box[aC] - Box[a ut C]) - C(z) (g_z Box[aS] - Box[a ut S]) ] }
// and dL/df(z) = T1(z) - alpha(z) E1(z); per-workgroup partial sums of
// alpha(x) E2(x) feed dL/dsigma_r.  SM >= 0 fixes a one-pass launch's chain
// start mode, as for the forward.
template <int SM = -1>
struct PolBackward {
    static constexpr int NCH = 4, NACC = 1, NAUX = 3, NRAW = 4, NPAIR = 2, NCTR = 2;
    static constexpr int START = SM;
    template <typename AT>
    __device__ static void kappa(const AT *aux, AT *k)
    {
        k[0] = aux[1];
        k[1] = aux[1] * aux[2];
    }
    template <typename AT>
    __device__ static AT ref(const IO &a, int i, int j)
    {
        return (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
    }
    template <typename AT>
    __device__ static void fetch(const IO &a, bool valid, int i, int j, AT *raw)
    {
        const long o = (long)i * a.W + j;
        const AT x0 = (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
        const AT x1 = (AT)a.aux0[o], x2 = (AT)a.aux1[o], x3 = (AT)a.aux2[o];
        raw[0] = valid ? x0 : AT(0);
        raw[1] = valid ? x1 : AT(0);
        raw[2] = valid ? x2 : AT(1);
        raw[3] = valid ? x3 : AT(0);
    }
    template <typename AT>
    __device__ static void make(const AT *raw, AT ref, AT *aux)
    {
        aux[0] = raw[0] - ref;
        // alpha = gbar / Q with the hardware reciprocal (about 1 ulp): three of these
        // per pixel and row, where an IEEE divide costs about ten instructions
        aux[1] = raw[1] * recip(raw[2]);
        aux[2] = raw[3] - ref;
    }
    template <typename AT>
    __device__ static void chans(AT C, AT S, const AT *aux, AT *X)
    {
        const AT aC = aux[1] * C, aS = aux[1] * S;
        X[0] = aC;
        X[1] = aS;
        X[2] = aux[2] * aC;
        X[3] = aux[2] * aS;
    }
    template <typename AT>
    __device__ static void recombine(AT v, AT vom, AT C, AT S, const AT *B, const AT *auxc, AT *acc)
    {
        // the same sum grouped by the centre's C and S:
        //   C (v Box[aC] + omega v (g_z Box[aS] - Box[a ut S]))
        // + S (v Box[aS] - omega v (g_z Box[aC] - Box[a ut C])),
        // six chained multiply-adds when v = 1 (the weight folded into the box sums)
        const AT gz = auxc[0];
        const AT t1 = fmat(gz, B[1], -B[3]);
        const AT t2 = fmat(gz, B[0], -B[2]);
        const AT u1 = fmat(vom, t1, v * B[0]);
        const AT u2 = fmat(-vom, t2, v * B[1]);
        acc[0] = fmat(C, u1, fmat(S, u2, acc[0]));
    }
    // the zero frequency: S = 0 and omega = 0, so only C(z) v Box[aC] remains
    template <typename AT>
    __device__ static void recombine_s0(AT v, AT C, const AT *B, AT *acc)
    {
        acc[0] = fmat(v * C, B[0], acc[0]);
    }
    // E1 and E2 of an output pixel, read only by its finalisation (the strip
    // body loads them a row ahead)
    template <typename AT>
    __device__ static void fetch_centre(const IO &a, int i, int j, AT *ctr)
    {
        const long o = (long)i * a.W + j;
        ctr[0] = (AT)a.aux3[o];
        ctr[1] = (AT)a.aux4[o];
    }
    template <typename AT>
    __device__ static void finalize(const IO &a, int i, int j, AT ref, const AT *auxc, const AT *acc,
                                    const AT *ctr, double *red)
    {
        const long o = (long)i * a.W + j;
        const AT alpha = auxc[1];
        if (a.out) ((float *)a.out)[o] = (float)(acc[0] - alpha * ctr[0]);
        *red += (double)alpha * (double)ctr[1];
    }
};
template <int SM>
struct FoldsWeight<PolBackward<SM>> {
    static constexpr bool value = true;
};

// ---------------------------------------------------------------- the body --
struct Geom {
    int H, W, pitch_in, pitch_out, rh, rv, S, K;   // K: padded to a multiple of KC
    int start_mode;    // first pass: 0 omega_0 = 0, 1 omega_0 = delta / 2, 2 general
    double omega_base, delta;
    const double *v;   // folded weights (FP64), K entries, zero past the kept orders
    const float *vf;   // the same weights in FP32
    void *ws;          // NACC planes of H*W accumulators, or null when K <= KC
    // separable spatial kernel (Algorithms 1 and 2 with M > 1): weight of the
    // zero frequency and of each spatial frequency, and the phase tables
    // (cos, sin)(nu_j y) per row and (cos, sin)(nu_j x) per column
    float sp_u0;
    float sp_u[kMaxSpatialFreq];
    const float *sp_row;
    const float *sp_col;
    // two-pixel patch: orders per first-pixel frequency (unpacked layout),
    // those frequencies, and the weights (device memory)
    int p2_group;
    double p2_omega1_base, p2_delta1;
    const float *p2_vf;
};

// Read-only tables read at workgroup-uniform addresses: through the constant
// address space the compiler fetches them with scalar loads into SGPRs
// instead of one vector load per lane.
template <typename AT>
using ConstPtr = const __attribute__((address_space(4))) AT *;

template <typename AT>
__device__ __forceinline__ AT weight(const Geom &gm, int m);
template <>
__device__ __forceinline__ float weight<float>(const Geom &gm, int m) { return gm.vf[m]; }
template <>
__device__ __forceinline__ double weight<double>(const Geom &gm, int m) { return gm.v[m]; }


// Two values of the compute type, moved between registers and LDS as one
// 64-bit (FP32) or 128-bit (FP64) access.
template <typename AT>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
    __device__ static float2 make(float a, float b) { return make_float2(a, b); }
};
template <>
struct Vec2<double> {
    using type = double2;
    __device__ static double2 make(double a, double b) { return make_double2(a, b); }
};

// Walker geometry of one LDS row of BLOCK columns.  The row holds column c at
// position c (a contiguous run of lanes touches distinct banks) and, after the
// H stage, the exclusive prefix sum E(c) = sum_{j < c} V(j), for c = 0 .. BLOCK.
// The two rows of a channel pair (the cosine and the sine member) are stored
// interleaved, element by element, so the V stage writes and the R stage reads
// both members with one wide access; a walker steps through its row with
// stride 2.
// CH walkers (a power of two, at most one wavefront) per row each own G
// consecutive positions, G odd: walker w starts at position G w, so the CH
// walkers of a row start on distinct banks, and rows in the same half
// wavefront are offset by RS = CH (mod 32) positions, which keeps their
// banks disjoint.  The last walker's chunk runs past position BLOCK into the
// row's tail; what it reads and writes there only feeds prefixes beyond BLOCK,
// which nothing uses.
constexpr int pow2_floor(int x) { return x >= 64 ? 64 : x >= 32 ? 32 : x >= 16 ? 16 : x >= 8 ? 8 : x >= 4 ? 4 : x >= 2 ? 2 : 1; }
constexpr int walker_count(int block, int rows) { return pow2_floor(block / rows); }
constexpr int walker_chunk(int block, int ch) { return (block / ch) % 2 == 0 ? block / ch + 1 : block / ch; }
constexpr int row_stride(int block, int ch, int g)
{
    int rs = ch * g > block + 1 ? ch * g : block + 1;
    if (ch < 32)
        while (rs % 32 != ch) ++rs;
    return rs;
}

// XCD-aware tile order.  The chip's 256 CUs sit in 8 XCDs, each with its own
// L2, and workgroups are dispatched to the XCDs round-robin by linear index.
// The strip kernels are launched one-dimensionally: workgroup L takes tile
// T = (L mod 8) * per + L / 8 (per = ceil(tiles / 8)), so each XCD works
// through a contiguous run of tiles, numbered strip-fastest (row-major over
// the segments).  Vertically adjacent segments, which share the 2r rows of
// the window, are then one row of tiles apart on the same XCD and resident
// together, and horizontally adjacent strips, which share the halo columns,
// are neighbours; each XCD still spans the image's whole width.  The up to
// seven workgroups past the last tile return at once.
constexpr int kXcd = 8;
__device__ __forceinline__ bool xcd_tile(int strips, int segs, int *bx, int *by)
{
    const int ntiles = strips * segs;
    const int per = (ntiles + kXcd - 1) / kXcd;
    const int L = blockIdx.x;
    const int T = (L % kXcd) * per + L / kXcd;
    if (T >= ntiles) return false;
    *by = T / strips;
    *bx = T - *by * strips;
    return true;
}
// Launch size of xcd_tile's grid for a strips x segs tiling.
inline unsigned xcd_grid(long long strips, long long segs)
{
    const long long ntiles = strips * segs;
    return (unsigned)(((ntiles + kXcd - 1) / kXcd) * kXcd);
}

// Floor division and the matching non-negative remainder, for the (possibly
// negative) interval offsets of the pipeline stages.
constexpr int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
constexpr int floormod(int a, int b) { return a - floordiv(a, b) * b; }

// LDS row buffers of the pipeline: the V stage fills one while the H stage
// scans the previous one and the R stage reads the one before that.
constexpr int kNBuf = 3;
// LDS rows per channel and order: 1 for the box; with the spatial kernel one
// row per horizontal basis function (the zero frequency when Ns is even, and
// a cosine and a sine row per non-zero frequency).
constexpr int spatial_rows(int nsc, bool even) { return nsc == 0 ? 1 : (even ? 1 : 0) + 2 * nsc; }
template <int NCH, int KL, int BLOCK, int NSC = 0, bool SEVEN = true>
constexpr int strip_lds_elems()
{
    constexpr int rows = NCH * KL * spatial_rows(NSC, SEVEN);
    return kNBuf * rows * row_stride(BLOCK, walker_count(BLOCK, rows), walker_chunk(BLOCK, walker_count(BLOCK, rows)));
}

// Exclusive prefix sums over aligned groups of CH consecutive lanes (CH a power
// of two, at most 64); wch is the lane's index in its group.  Groups of 16 are
// DPP rows: four shifted adds within the row and one final shift, no LDS.
// Lane l - N of the same 16-lane DPP row (zero for the row's first N lanes);
// N = 0 is the lane itself.
template <int N>
__device__ __forceinline__ float dpp_row_shr(float x)
{
    static_assert(N >= 0 && N <= 15, "row_shr reaches 15 lanes");
    if constexpr (N == 0) return x;
    else return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + N, 0xf, 0xf, true));
}

// A DPP lane move of a 64-bit value: both 32-bit halves with the same control;
// lanes that the control leaves without a source (or rows outside row_mask)
// read zero.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int CH, typename AT>
__device__ __forceinline__ AT group_exclusive_scan(AT x, int wch)
{
    if constexpr ((CH == 16 || CH == 32) && sizeof(AT) == 8) {
        // FP64: the same row scans on the two halves; groups of 32 add the last
        // lane of the lower row to the upper one (row_bcast:15, rows 1 and 3)
        // and shift across the row boundary (wave_shr:1, zero at a group's first lane)
        double y = x;
        y += dpp64<0x111, 0xf>(y);
        y += dpp64<0x112, 0xf>(y);
        y += dpp64<0x114, 0xf>(y);
        y += dpp64<0x118, 0xf>(y);
        if constexpr (CH == 16) {
            return dpp64<0x111, 0xf>(y);
        } else {
            y += dpp64<0x142, 0xa>(y);
            const double e = dpp64<0x138, 0xf>(y);
            return wch == 0 ? 0.0 : e;
        }
    } else if constexpr (CH == 16 && sizeof(AT) == 4) {
        // row_shr:n (dpp_ctrl 0x110 + n) reads lane l - n of the same row; the
        // first n lanes of the row read zero (bound_ctrl)
        float y = x;
        y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x111, 0xf, 0xf, true));
        y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x112, 0xf, 0xf, true));
        y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x114, 0xf, 0xf, true));
        y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x118, 0xf, 0xf, true));
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x111, 0xf, 0xf, true));
    } else {
        // inclusive scan, then a shift by one lane (never inc - x: the last
        // walker's total includes the unused tail of the row)
        AT inc = x;
#pragma unroll
        for (int d = 1; d < CH; d <<= 1) {
            const AT y = __shfl_up(inc, d, CH);
            if (wch >= d) inc += y;
        }
        const AT prev = __shfl_up(inc, 1, CH);
        return wch > 0 ? prev : AT(0);
    }
}

// The strip body, software-pipelined over "intervals" of KL orders of one row.
// Interval t runs three stages on three LDS row buffers (t mod 3):
//   V (interval t)      vertical moving sums of the KL orders, written to buffer t;
//   H (interval t - 1)  the walkers turn buffer t - 1 into prefix sums in place;
//   R (interval t - 2)  output lanes read box sums from buffer t - 2 and
//                       recombine them with the centre pixel's transforms;
// then one workgroup barrier.  The stages touch different buffers, so each
// interval mixes the VALU-heavy V stage with the LDS-heavy H and R stages.
// KR orders are carried in registers per pass (the vertical sums of all their
// channels), NSUB = KR / KL intervals per row.
//
// With NSC > 0 the spatial kernel is the separable raised cosine
// w(dy) w(dx), w(d) = u0 + sum_j u_j cos(nu_j d) (u0 = 0 unless SEVEN), rather
// than the box.  The vertical factor is exact in the V stage: next to the plain
// moving sum V, each channel keeps per frequency the running sum
// W_j = sum_{y in window} e^{i nu_j y} X(y) (absolute rows, so the update needs
// no rotation), and the row written to LDS is the weighted vertical sum
// VQ(i) = u0 V + sum_j Re(e^{-i nu_j i} W_j).  The horizontal factor uses the
// shift identity along the row: VQ, VQ cos(nu_j x) and VQ sin(nu_j x) are
// prefix-summed, and the R stage forms
// u0 Box[VQ] + sum_j u_j (cos(nu_j x) Box[VQ cos] + sin(nu_j x) Box[VQ sin]).
//
// RHC > 0 fixes the horizontal radius at compile time (rh == RHC).  The
// one-pass plain FP32 forward then has its walkers hand out box sums rather
// than prefix sums: a walker holds the prefixes E of its G positions in
// registers, and E(p - 2 rh - 1) lies a fixed number of walkers to the left in
// the same DPP row (the shift and the element index follow from 2 rh + 1 and
// G), so each box sum Box(p) = E(p) - E(p - 2 rh - 1) costs one DPP-shifted
// subtraction and the R stage reads one value per channel instead of two.
template <typename AT, int BLOCK, int KR, int KL, class POL, int QUANT, bool KAHAN, int NSC = 0,
          bool SEVEN = true, int RHC = 0>
__device__ __forceinline__ void strip_body(const IO &a, const Geom &gm, int bx, int by, AT *lds,
                                           double *red_lds, double *red_out)
{
    constexpr int NCH = POL::NCH;
    constexpr int NACC = POL::NACC;
    constexpr int NAUX = POL::NAUX;
    constexpr int NRAW = POL::NRAW;
    constexpr int NPAIR = POL::NPAIR;
    constexpr int NB = spatial_rows(NSC, SEVEN);
    constexpr bool PLAIN = NSC == 0 || SEVEN;   // the zero spatial frequency is present
    constexpr int NSCR = NSC > 0 ? NSC : 1;      // array extent
    constexpr int ROWS = NCH * KL * NB;
    constexpr int CH = walker_count(BLOCK, ROWS);
    constexpr int G = walker_chunk(BLOCK, CH);
    constexpr int RS = row_stride(BLOCK, CH, G);
    constexpr int BUF = ROWS * RS;
    constexpr int NSUB = KR / KL;
    static_assert(NCH == 2 * NPAIR, "channels come in (cos, sin) pairs");
    static_assert(KR % KL == 0, "KR must be a multiple of KL");
    static_assert(CH * G >= BLOCK + 1 && RS >= CH * G && ROWS * CH <= BLOCK, "walker geometry");
    static_assert(NSC <= kMaxSpatialFreq && (NSC == 0 || (!KAHAN && sizeof(AT) == 4)),
                  "the spatial kernel runs the plain FP32 forward");

    const int t = threadIdx.x;
    const int H = gm.H, W = gm.W, rh = RHC > 0 ? RHC : gm.rh, rv = gm.rv;
    const int Wt = BLOCK - 2 * rh;
    const int j0 = bx * Wt;
    const int jx = j0 - rh + t;
    const bool colok = (jx >= 0) && (jx < W);
    const int i0 = by * gm.S;
    const int i1 = min(H, i0 + gm.S);
    const int ylo = max(0, i0 - rv);
    const int yhi = min(H, i0 + rv);
    const bool outlane = (t >= rh) && (t < rh + Wt) && colok;
    const AT ref = POL::template ref<AT>(a, i0, min(W - 1, j0 + Wt / 2));
    const long plane = (long)H * W;

    // LDS positions: this lane's column (V stage), its walker chunk (H stage),
    // and the two prefix positions its output needs (R stage).  Rows are
    // clamped into the image and columns to jxc so that every load is to an
    // in-image address; absent pixels are masked by the policies' fetch.
    const int jxc = min(max(jx, 0), W - 1);
    auto rowc = [H](int y) { return min(max(y, 0), H - 1); };
    const int vpos = t;
    const int wrow = t / CH;
    const int wch = t - wrow * CH;
    constexpr bool ALLWALK = ROWS * CH == BLOCK;
    const bool walker = ALLWALK || wrow < ROWS;
    // FP32: row r of a buffer is member (r & 1) of pair-row r >> 1, the two
    // members interleaved (element u of this walker's chunk at wbase + 2 u).
    // FP64 keeps every row contiguous (element u at wbase + u): interleaved
    // 8-byte members would put walkers 8 apart on the same banks, while with
    // G odd the walkers of a contiguous row start on distinct bank pairs.
    constexpr bool PAIRED = sizeof(AT) == 4;
    constexpr int WST = PAIRED ? 2 : 1;
    const int wbase = PAIRED ? (wrow >> 1) * (2 * RS) + 2 * (wch * G) + (wrow & 1) : wrow * RS + wch * G;
    using V2 = typename Vec2<AT>::type;
    // box sum of output lane t: E(t + rh + 1) - E(t - rh)
    const int phi = t + rh + 1;
    const int plo = t - rh;

    // spatial kernel: this column's horizontal basis values (V stage) and the
    // output column's coefficients u_j (cos, sin)(nu_j x) (R stage)
    float hc[NSCR], hs[NSCR], rcw[NSCR], rsw[NSCR];
    const float u0 = NSC > 0 ? gm.sp_u0 : 1.0f;
#pragma unroll
    for (int j = 0; j < NSCR; ++j) {
        hc[j] = hs[j] = rcw[j] = rsw[j] = 0.0f;
        if constexpr (NSC > 0) {
            hc[j] = gm.sp_col[2 * ((long)j * W + jxc)];
            hs[j] = gm.sp_col[2 * ((long)j * W + jxc) + 1];
            rcw[j] = gm.sp_u[j] * hc[j];
            rsw[j] = gm.sp_u[j] * hs[j];
        }
    }
    // (cos, sin)(nu_j y) of image row y, uniform over the workgroup
    auto phase = [&](int j, int y, float *c, float *s) {
        *c = gm.sp_row[2 * ((long)j * H + y)];
        *s = gm.sp_row[2 * ((long)j * H + y) + 1];
    };

    double red = 0.0;

    // The order of this lane's walker row within an interval: rows are ordered
    // (order k, pair, horizontal basis row, member), NCH NB rows per order.
    // When the rows of one wavefront all belong to one order the index is made
    // wave-uniform, so that the weights come from scalar loads.
    // (the patch kernels fold their weights only where the walkers form box
    // sums: with the run-time radius the fold measured 0.7% slower there)
    constexpr bool FOLDV = FoldsWeight<POL>::value && (!IsPatch2<POL>::value || RHC > 0);
    constexpr int RPW = 64 / CH;   // walker rows per wavefront
    int kw = min(wrow, ROWS - 1) / (NCH * NB);
    if constexpr (RPW <= NCH * NB && (NCH * NB) % RPW == 0) kw = __builtin_amdgcn_readfirstlane(kw);

    // POL::START >= 0: one pass (K <= KR) whose chain start mode is that constant
    constexpr int CSTART = POL::START;
    const int Kloop = CSTART >= 0 ? 1 : gm.K;
    // Order m of a one-pass launch with the chain start of even N is the zero
    // frequency: its sine channels vanish identically, so their sums, updates
    // and recombination terms are skipped (m is a constant of the unrolled loops).
    auto zero_sine = [](int m) { return CSTART == 0 && m == 0; };
    for (int m0 = 0; m0 < Kloop; m0 += KR) {
        const bool first = (m0 == 0);
        const bool last = CSTART >= 0 || (m0 + KR >= gm.K);
        AT om0 = (AT)(gm.omega_base + (double)m0 * gm.delta);
        const AT dlt = (AT)gm.delta;
        const int smode = first ? (CSTART >= 0 ? CSTART : gm.start_mode) : 2;
        AT om1 = AT(0), d1 = AT(0);
        if constexpr (IsPatch2<POL>::value) {
            // the first-pixel frequency of the pass's first order and the second
            // pixel's frequency of that order: either the pass holds KR / G whole
            // groups, each from the second pixel's first order, or it lies within
            // one group of p2_group orders
            int n1;
            if constexpr (POL::GROUP > 0) {
                n1 = (m0 / KR) * (KR / POL::GROUP);
                om0 = (AT)gm.omega_base;
            } else {
                n1 = m0 / gm.p2_group;
                om0 = (AT)(gm.omega_base + (double)(m0 - n1 * gm.p2_group) * gm.delta);
            }
            om1 = (AT)(gm.p2_omega1_base + (double)n1 * gm.p2_delta1);
            d1 = (AT)gm.p2_delta1;
        }

        // weights of the walker rows of each sub-phase (FOLDV)
        AT vH[FOLDV ? NSUB : 1];
#pragma unroll
        for (int s = 0; s < (FOLDV ? NSUB : 1); ++s) {
            if constexpr (!FOLDV) vH[s] = AT(1);
            else if constexpr (IsPatch2<POL>::value) vH[s] = ((ConstPtr<float>)gm.p2_vf)[m0 + s * KL + kw];
            else vH[s] = weight<AT>(gm, m0 + s * KL + kw);
        }

        AT V[KR][NCH];
        AT Cmp[KAHAN ? KR : 1][NCH];
        AT Wr[NSC > 0 ? KR : 1][NCH][NSCR], Wi[NSC > 0 ? KR : 1][NCH][NSCR];
#pragma unroll
        for (int m = 0; m < KR; ++m)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                V[m][ch] = AT(0);
                Cmp[KAHAN ? m : 0][ch] = AT(0);
#pragma unroll
                for (int j = 0; j < NSCR; ++j) Wr[NSC > 0 ? m : 0][ch][j] = Wi[NSC > 0 ? m : 0][ch][j] = AT(0);
            }

        // initial window: rows [i0 - rv, i0 + rv - 1] (the first step adds i0 + rv)
        {
            AT raw[NRAW];
            POL::template fetch<AT>(a, colok, rowc(ylo), jxc, raw);
            for (int y = ylo; y < yhi; ++y) {
                AT aux[NAUX], kp[NPAIR];
                POL::template make<AT>(raw, ref, aux);
                POL::template kappa<AT>(aux, kp);
                POL::template fetch<AT>(a, colok, rowc(y + 1), jxc, raw);
                AT kc[NPAIR][NSCR], ks[NPAIR][NSCR];
                if constexpr (NSC > 0) {
#pragma unroll
                    for (int j = 0; j < NSC; ++j) {
                        float c, s;
                        phase(j, y, &c, &s);
#pragma unroll
                        for (int p = 0; p < NPAIR; ++p) {
                            kc[p][j] = kp[p] * c;
                            ks[p][j] = kp[p] * s;
                        }
                    }
                }
                typename ChainOf<POL, AT>::type ch;
                chain_start<POL>(ch, colok, aux, om0, dlt, smode, om1, d1);
#pragma unroll
                for (int m = 0; m < KR; ++m) {
                    const bool zs = zero_sine(m);
                    chain_restart<POL>(ch, m);
                    const AT C = quant<QUANT>(ch.c), S = quant<QUANT>(ch.s);
#pragma unroll
                    for (int p = 0; p < NPAIR; ++p) {
                        if constexpr (PLAIN) {
                            V[m][2 * p] = fmat(kp[p], C, V[m][2 * p]);
                            if (!zs) V[m][2 * p + 1] = fmat(kp[p], S, V[m][2 * p + 1]);
                        }
                        if constexpr (NSC > 0) {
#pragma unroll
                            for (int j = 0; j < NSC; ++j) {
                                Wr[m][2 * p][j] = fmat(kc[p][j], C, Wr[m][2 * p][j]);
                                Wi[m][2 * p][j] = fmat(ks[p][j], C, Wi[m][2 * p][j]);
                                Wr[m][2 * p + 1][j] = fmat(kc[p][j], S, Wr[m][2 * p + 1][j]);
                                Wi[m][2 * p + 1][j] = fmat(ks[p][j], S, Wi[m][2 * p + 1][j]);
                            }
                        }
                    }
                    if (zs) ch.template step<true>();
                    else ch.step();
                }
            }
        }

        // raw inputs fetched one row ahead: incoming and outgoing rows for the
        // V stage, the centre row for the R stage
        AT rin[NRAW], rout[NRAW], rc[NRAW];
        {
            const int yin = i0 + rv, yout = i0 - rv - 1;
            POL::template fetch<AT>(a, colok && yin < H, rowc(yin), jxc, rin);
            POL::template fetch<AT>(a, colok && yout >= ylo, rowc(yout), jxc, rout);
            POL::template fetch<AT>(a, colok, i0, jxc, rc);
        }
        typename ChainOf<POL, AT>::type ci, co, cc;
        AT ki[NPAIR], ko[NPAIR], auxc[NAUX], acc[NACC];
        // a later pass's partial accumulators of the R stage's row, read from the
        // workspace when the row's R stage starts, added when it ends (NSUB
        // intervals later), so the HBM latency is not waited out at the row's end
        AT wsv[NACC];
#pragma unroll
        for (int q = 0; q < NACC; ++q) wsv[q] = AT(0);
        // per-pixel inputs that only the last pass's finalisation reads, loaded
        // one row ahead for the same reason
        constexpr int NCTR = POL::NCTR;
        AT ctr[NCTR > 0 ? NCTR : 1];
#pragma unroll
        for (int q = 0; q < (NCTR > 0 ? NCTR : 1); ++q) ctr[q] = AT(0);
        if constexpr (NCTR > 0) {
            if (last && outlane) POL::template fetch_centre<AT>(a, i0, jx, ctr);
        }
        // spatial kernel: kappa times the phases of the incoming and outgoing
        // rows, and u_j (cos, sin)(nu_j i) of the output row
        AT kic[NPAIR][NSCR], kis[NPAIR][NSCR], koc[NPAIR][NSCR], kos[NPAIR][NSCR];
        AT dc[NSCR], ds[NSCR];
#pragma unroll
        for (int j = 0; j < NSCR; ++j) {
            dc[j] = ds[j] = AT(0);
#pragma unroll
            for (int p = 0; p < NPAIR; ++p) kic[p][j] = kis[p][j] = koc[p][j] = kos[p][j] = AT(0);
        }
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) ki[p] = ko[p] = AT(0);
#pragma unroll
        for (int q = 0; q < NAUX; ++q) auxc[q] = AT(0);
#pragma unroll
        for (int q = 0; q < NACC; ++q) acc[q] = AT(0);
        int bv = 0;

        // Interval (i, h): the V stage of sub-phase h of row i, the H stage one
        // interval behind and the R stage two behind; the last interval with
        // work is (i1 - i0) NSUB + 1.
        const int iend = i1 + (NSUB >= 2 ? 1 : 2);
        for (int i = i0; i < iend; ++i) {
#pragma unroll
            for (int h = 0; h < NSUB; ++h) {
                const int iH = i + floordiv(h - 1, NSUB);
                const int iR = i + floordiv(h - 2, NSUB);
                const int sR = floormod(h - 2, NSUB);
                const bool actV = i < i1;
                const bool actH = iH >= i0 && iH < i1;
                const bool actR = iR >= i0 && iR < i1;
                // intervals past the last one with work do nothing (uniform)
                if (!(actV || actH || actR)) continue;
                const int bH = bv == 0 ? kNBuf - 1 : bv - 1;
                const int bR = bH == 0 ? kNBuf - 1 : bH - 1;
                V2 *const VbV = reinterpret_cast<V2 *>(lds + bv * BUF);
                AT *const VbH = lds + bH * BUF;
                const V2 *const VbR = reinterpret_cast<const V2 *>(lds + bR * BUF);

                // Wave priorities per stage (H above R above V): a SIMD's arbiter then
                // issues the LDS-bound stages of the waves that have just passed the
                // barrier ahead of the VALU-bound V stage of the others, so the
                // barrier's critical path shortens while V fills the gaps.
                __builtin_amdgcn_s_setprio(1);
                // One-pass plain FP32 forward on the box path: the R stage's box-sum
                // prefixes and the walker's chunk are read together, right after the
                // barrier, so the two LDS latencies overlap.  That is 1% faster there;
                // the multi-pass and 16-bit-stack forwards and the policies with more
                // channels or two values per pixel measured slower with it.
                constexpr bool JOINT = NSC == 0 && IsForward32<POL>::value && POL::START >= 0 && QUANT == 0 &&
                                       !KAHAN;
                constexpr int NRD = JOINT ? KL * NPAIR : 1;
                // walkers that produce box sums: one DPP row per LDS row, and the
                // source walker at most 15 lanes to the left
                constexpr bool WBOX = RHC > 0 && PAIRED && FOLDV && CH == 16 && (2 * RHC + 1) / G + 1 <= 15;
                V2 rhi[NRD], rlo[NRD];
                AT loc[G];
                if constexpr (JOINT) {
                    if (actR && outlane) {
#pragma unroll
                        for (int q = 0; q < NRD; ++q) {
                            rhi[q] = VbR[q * RS + phi];
                            if constexpr (!WBOX) rlo[q] = VbR[q * RS + plo];
                        }
                    }
                    // Read whether or not the H stage runs this interval (every lane of
                    // this launch shape is a walker and its chunk lies inside the
                    // buffer): a conditional read would make loc[] a value carried
                    // from one interval to the next, which the compiler keeps with
                    // a register copy per element.
                    static_assert(!JOINT || ALLWALK, "joint reads assume every lane walks");
#pragma unroll
                    for (int u = 0; u < G; ++u) loc[u] = VbH[wbase + WST * u];
                }
                // ---- R stage: box sums of the orders sR KL .. of row iR, recombined
                if (actR && outlane) {
                    if (sR == 0) {
                        POL::template make<AT>(rc, ref, auxc);
                        POL::template fetch<AT>(a, colok, rowc(iR + 1), jxc, rc);
                        chain_start<POL>(cc, colok, auxc, om0, dlt, smode, om1, d1);
#pragma unroll
                        for (int q = 0; q < NACC; ++q) acc[q] = AT(0);
                        if (!first) {
                            const long o = (long)iR * W + jx;
#pragma unroll
                            for (int q = 0; q < NACC; ++q) wsv[q] = ((const AT *)gm.ws)[q * plane + o];
                        }
                    }
#pragma unroll
                    for (int k = 0; k < KL; ++k) {
                        const int m = sR * KL + k;
                        AT B[NCH];
#pragma unroll
                        for (int p = 0; p < NPAIR; ++p) {
                            // pair-row of channels (2p, 2p + 1), horizontal basis function b
                            const V2 *prow = VbR + (k * NPAIR + p) * NB * RS;
                            if constexpr (WBOX && JOINT) {
                                // the box sums themselves, read at position phi after the barrier
                                B[2 * p] = rhi[k * NPAIR + p].x;
                                B[2 * p + 1] = rhi[k * NPAIR + p].y;
                            } else if constexpr (JOINT) {
                                const V2 hi = rhi[k * NPAIR + p], lo = rlo[k * NPAIR + p];
                                B[2 * p] = hi.x - lo.x;
                                B[2 * p + 1] = hi.y - lo.y;
                            } else if constexpr (WBOX && NSC == 0) {
                                // the box sums themselves, stored at position phi
                                const V2 hi = prow[phi];
                                B[2 * p] = hi.x;
                                B[2 * p + 1] = hi.y;
                            } else if constexpr (NSC == 0 && PAIRED) {
                                const V2 hi = prow[phi], lo = prow[plo];
                                B[2 * p] = hi.x - lo.x;
                                B[2 * p + 1] = hi.y - lo.y;
                            } else if constexpr (NSC == 0) {
                                // contiguous rows 2 (k NPAIR + p) and the next one
                                const AT *r0 = reinterpret_cast<const AT *>(VbR) + 2 * (k * NPAIR + p) * RS;
                                B[2 * p] = r0[phi] - r0[plo];
                                B[2 * p + 1] = r0[RS + phi] - r0[RS + plo];
                            } else {
                                // box sums of a basis row pair: from two prefixes, or the
                                // walkers' box sum itself
                                auto box = [&](const V2 *row) {
                                    if constexpr (WBOX) {
                                        return row[phi];
                                    } else {
                                        const V2 hi = row[phi], lo = row[plo];
                                        return Vec2<AT>::make(hi.x - lo.x, hi.y - lo.y);
                                    }
                                };
                                AT h0 = AT(0), h1 = AT(0);
                                int b = 0;
                                if constexpr (SEVEN) {
                                    const V2 bz = box(prow);
                                    h0 = u0 * bz.x;
                                    h1 = u0 * bz.y;
                                    b = 1;
                                }
#pragma unroll
                                for (int j = 0; j < NSC; ++j) {
                                    const V2 *rc_ = prow + (b + 2 * j) * RS;
                                    const V2 bc = box(rc_), bs = box(rc_ + RS);
                                    h0 = fmat(rsw[j], bs.x, fmat(rcw[j], bc.x, h0));
                                    h1 = fmat(rsw[j], bs.y, fmat(rcw[j], bc.y, h1));
                                }
                                B[2 * p] = h0;
                                B[2 * p + 1] = h1;
                            }
                        }
                        chain_restart<POL>(cc, m);
                        AT v;
                        if constexpr (FOLDV) v = AT(1);   // already in B
                        else if constexpr (IsPatch2<POL>::value) v = ((ConstPtr<float>)gm.p2_vf)[m0 + m];
                        else v = weight<AT>(gm, m0 + m);
                        const AT vom = v * (om0 + (AT)m * dlt);
                        if constexpr (CSTART == 0) {
                            if (zero_sine(m)) {
                                POL::template recombine_s0<AT>(v, quant<QUANT>(cc.c), B, acc);
                                cc.template step<true>();
                                continue;
                            }
                        }
                        POL::template recombine<AT>(v, vom, quant<QUANT>(cc.c), quant<QUANT>(cc.s), B, auxc, acc);
                        cc.step();
                    }
                }

                __builtin_amdgcn_s_setprio(2);
                // ---- H stage: every row of buffer t - 1 into its exclusive prefix sums, in place
                if (actH) {
                    AT run = AT(0);
                    if (walker) {
                        if constexpr (!JOINT) {
#pragma unroll
                            for (int u = 0; u < G; ++u) loc[u] = VbH[wbase + WST * u];
                        }
                        // local exclusive prefixes: loc[u] = sum_{v < u} of the chunk (loc[0] = 0 is implicit)
                        run = loc[0];
#pragma unroll
                        for (int u = 1; u < G; ++u) {
                            const AT x = loc[u];
                            loc[u] = run;
                            run += x;
                        }
                    }
                    const AT off = group_exclusive_scan<CH>(run, wch);
                    if (walker) {
                        if constexpr (FOLDV) {
                            // the prefixes of order m scaled by its weight v_m
                            const AT vw = vH[floormod(h - 1, NSUB)];
                            // box-sum walkers: a multiply-add with a zero addend is the
                            // rounded product, and keeps the compiler from fusing it into
                            // the box subtraction below (E(p) - E(p - D) at u = 0), so the
                            // box sums are the same subtractions of the same prefix values
                            // that the run-time-radius kernels make in their R stage
                            AT offv;
                            if constexpr (WBOX) offv = fmat(off, vw, AT(0));
                            else offv = off * vw;
                            if constexpr (WBOX) {
                                // position p = G w + u: E(p - D), D = 2 rh + 1, is element
                                // u - D mod G of walker w - QS (u >= DR) or of walker
                                // w - QS - 1 (u < DR); positions below D (no output
                                // reads them) take a zero from the DPP bound control
                                constexpr int D = 2 * RHC + 1, QS = D / G, DR = D % G;
                                AT E[G];
                                E[0] = offv;
#pragma unroll
                                for (int u = 1; u < G; ++u) E[u] = fmat(loc[u], vw, offv);
#pragma unroll
                                for (int u = 0; u < G; ++u) {
                                    const AT lo = u >= DR ? dpp_row_shr<QS>(E[u >= DR ? u - DR : 0])
                                                          : dpp_row_shr<QS + 1>(E[u < DR ? u - DR + G : 0]);
                                    VbH[wbase + WST * u] = E[u] - lo;
                                }
                            } else {
                                VbH[wbase] = offv;
#pragma unroll
                                for (int u = 1; u < G; ++u) VbH[wbase + WST * u] = fmat(loc[u], vw, offv);
                            }
                        } else {
                            VbH[wbase] = off;
#pragma unroll
                            for (int u = 1; u < G; ++u) VbH[wbase + WST * u] = loc[u] + off;
                        }
                    }
                }

                __builtin_amdgcn_s_setprio(0);
                // ---- V stage: vertical moving sums V += X(i + rv) - X(i - rv - 1)
                if (actV) {
                    if (h == 0) {
                        const int yin = i + rv, yout = i - rv - 1;
                        const bool vin = colok && (yin < H);
                        const bool vout = colok && (yout >= ylo);
                        AT auxi[NAUX], auxo[NAUX];
                        POL::template make<AT>(rin, ref, auxi);
                        POL::template make<AT>(rout, ref, auxo);
                        POL::template kappa<AT>(auxi, ki);
                        POL::template kappa<AT>(auxo, ko);
                        POL::template fetch<AT>(a, colok && yin + 1 < H, rowc(yin + 1), jxc, rin);
                        POL::template fetch<AT>(a, colok && yout + 1 >= ylo, rowc(yout + 1), jxc, rout);
                        chain_start<POL>(ci, vin, auxi, om0, dlt, smode, om1, d1);
                        chain_start<POL>(co, vout, auxo, om0, dlt, smode, om1, d1);
                        if constexpr (NSC > 0) {
#pragma unroll
                            for (int j = 0; j < NSC; ++j) {
                                float c1, s1, c2, s2, c3, s3;
                                phase(j, rowc(yin), &c1, &s1);
                                phase(j, rowc(yout), &c2, &s2);
                                phase(j, i, &c3, &s3);
                                dc[j] = gm.sp_u[j] * c3;
                                ds[j] = gm.sp_u[j] * s3;
#pragma unroll
                                for (int p = 0; p < NPAIR; ++p) {
                                    kic[p][j] = ki[p] * c1;
                                    kis[p][j] = ki[p] * s1;
                                    koc[p][j] = ko[p] * c2;
                                    kos[p][j] = ko[p] * s2;
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < KL; ++k) {
                        const int m = h * KL + k;
                        chain_restart<POL>(ci, m);
                        chain_restart<POL>(co, m);
                        const AT Ci = quant<QUANT>(ci.c), Si = quant<QUANT>(ci.s);
                        const AT Co = quant<QUANT>(co.c), So = quant<QUANT>(co.s);
                        const bool zs = zero_sine(m);
#pragma unroll
                        for (int p = 0; p < NPAIR; ++p) {
                            if constexpr (KAHAN) {
                                const AT x[2] = {ki[p] * Ci - ko[p] * Co, ki[p] * Si - ko[p] * So};
#pragma unroll
                                for (int e = 0; e < (zs ? 1 : 2); ++e) {
                                    const int c = 2 * p + e;
                                    const AT y = x[e] - Cmp[m][c];
                                    const AT s = V[m][c] + y;
                                    Cmp[m][c] = (s - V[m][c]) - y;
                                    V[m][c] = s;
                                }
                            } else {
                                if constexpr (PLAIN) {
                                    V[m][2 * p] = fmat(-ko[p], Co, fmat(ki[p], Ci, V[m][2 * p]));
                                    if (!zs) V[m][2 * p + 1] = fmat(-ko[p], So, fmat(ki[p], Si, V[m][2 * p + 1]));
                                }
                                if constexpr (NSC > 0) {
#pragma unroll
                                    for (int j = 0; j < NSC; ++j) {
                                        AT *wr0 = &Wr[m][2 * p][j], *wi0 = &Wi[m][2 * p][j];
                                        AT *wr1 = &Wr[m][2 * p + 1][j], *wi1 = &Wi[m][2 * p + 1][j];
                                        *wr0 = fmat(-koc[p][j], Co, fmat(kic[p][j], Ci, *wr0));
                                        *wi0 = fmat(-kos[p][j], Co, fmat(kis[p][j], Ci, *wi0));
                                        *wr1 = fmat(-koc[p][j], So, fmat(kic[p][j], Si, *wr1));
                                        *wi1 = fmat(-kos[p][j], So, fmat(kis[p][j], Si, *wi1));
                                    }
                                }
                            }
                        }
#pragma unroll
                        for (int p = 0; p < NPAIR; ++p) {
                            V2 *prow = VbV + (k * NPAIR + p) * NB * RS + vpos;
                            if constexpr (NSC == 0 && PAIRED) {
                                prow[0] = Vec2<AT>::make(V[m][2 * p], V[m][2 * p + 1]);
                            } else if constexpr (NSC == 0) {
                                AT *r0 = reinterpret_cast<AT *>(VbV) + 2 * (k * NPAIR + p) * RS + vpos;
                                r0[0] = V[m][2 * p];
                                r0[RS] = V[m][2 * p + 1];
                            } else {
                                // vertically weighted sums of the pair, then their horizontal basis rows
                                AT vq[2];
#pragma unroll
                                for (int e = 0; e < 2; ++e) {
                                    const int c = 2 * p + e;
                                    vq[e] = PLAIN ? u0 * V[m][c] : AT(0);
#pragma unroll
                                    for (int j = 0; j < NSC; ++j)
                                        vq[e] = fmat(ds[j], Wi[m][c][j], fmat(dc[j], Wr[m][c][j], vq[e]));
                                }
                                int b = 0;
                                if constexpr (SEVEN) {
                                    prow[0] = Vec2<AT>::make(vq[0], vq[1]);
                                    b = 1;
                                }
#pragma unroll
                                for (int j = 0; j < NSC; ++j) {
                                    prow[(b + 2 * j) * RS] = Vec2<AT>::make(vq[0] * hc[j], vq[1] * hc[j]);
                                    prow[(b + 2 * j + 1) * RS] = Vec2<AT>::make(vq[0] * hs[j], vq[1] * hs[j]);
                                }
                            }
                        }
                        if (zs) {
                            ci.template step<true>();
                            co.template step<true>();
                        } else {
                            ci.step();
                            co.step();
                        }
                    }
                }

                // ---- row iR complete: continue or finish its accumulators
                if (actR && sR == NSUB - 1 && outlane) {
                    const long o = (long)iR * W + jx;
                    if (!first) {
#pragma unroll
                        for (int q = 0; q < NACC; ++q) acc[q] += wsv[q];
                    }
                    if (last) {
                        if constexpr (QUANT != 0 && IsForward32<POL>::value) {
                            // 16-bit stacks: the exact normaliser is at least the kernel's
                            // centre value (about 1) for a non-negative kernel; one that fell
                            // below 1/2 is dominated by quantisation error, and the pixel
                            // keeps its own value instead of an unbounded ratio
                            if (!(acc[0] >= AT(0.5))) {
                                acc[0] = AT(1);
                                acc[1] = auxc[0];
                            }
                        }
                        POL::template finalize<AT>(a, iR, jx, ref, auxc, acc, ctr, &red);
                        if constexpr (NCTR > 0) POL::template fetch_centre<AT>(a, rowc(iR + 1), jx, ctr);
                    } else {
#pragma unroll
                        for (int q = 0; q < NACC; ++q) ((AT *)gm.ws)[q * plane + o] = acc[q];
                    }
                }
                __syncthreads();
                bv = bv == kNBuf - 1 ? 0 : bv + 1;
            }
        }
    }

    if (red_out) {
        // deterministic block reduction (fixed order) of the per-lane sums; the
        // barrier first, as red_lds may alias the row buffers
        __syncthreads();
        red_lds[t] = red;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int q = 0; q < BLOCK; ++q) s += red_lds[q];
            *red_out = s;
        }
        __syncthreads();
    }
}

}  // namespace bsk
