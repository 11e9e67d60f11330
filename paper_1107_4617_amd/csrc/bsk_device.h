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
// column j0 - rh + t.  Per output row i:
//   phase V  every lane updates, in registers, the vertical moving sums of all
//            channels of its column for the chunk's KC orders:
//            V += X(i + rv) - X(i - rv - 1).  The transforms X come from a
//            rotation recurrence over the orders (one sincos pair per pixel,
//            then a 2x2 rotation per order), so cos/sin are never evaluated
//            per order.  V is written to an LDS row buffer.
//   phase H  "walker" lanes, one per (order, channel, segment of columns),
//            slide a horizontal window of width 2 rh + 1 along the LDS row:
//            B(j) = B(j - 1) + V(j + rh) - V(j - rh - 1).
//   phase R  every output lane recombines its pixel from the box sums of all
//            orders and the transforms of its own value (kept in registers).
// The (channels x orders) stack therefore lives only in registers and LDS; HBM
// sees the input (read ~3 times through L2: as incoming, centre and outgoing
// row) and the output.  Values are centred on a per-workgroup reference level
// before transforming (the filter is shift covariant), which halves the
// magnitude of the f-weighted sums.  Orders beyond KC are processed in further
// passes whose partial accumulators live in a workspace.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "bsk_internal.h"

namespace bsk {

// ------------------------------------------------------------------ helpers --
__device__ __forceinline__ void sc(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void sc(double x, double *s, double *c) { sincos(x, s, c); }

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

template <typename AT>
struct Chain {
    AT c, s, cd, sd;
    // (c, s) = (cos, sin)(om0 g), rotation step (cos, sin)(dlt g); a pixel
    // outside the image starts at (0, 0) so all its channels vanish.
    __device__ __forceinline__ void start(bool valid, AT g, AT om0, AT dlt)
    {
        AT s0, c0, s1, c1;
        sc(om0 * g, &s0, &c0);
        sc(dlt * g, &s1, &c1);
        c = valid ? c0 : AT(0);
        s = valid ? s0 : AT(0);
        cd = c1;
        sd = s1;
    }
    __device__ __forceinline__ void step()
    {
        const AT cn = c * cd - s * sd;
        const AT sn = s * cd + c * sd;
        c = cn;
        s = sn;
    }
};

template <typename T>
__device__ __forceinline__ T ld(const void *p, long idx) { return ((const T *)p)[idx]; }

// ------------------------------------------------------------------ policies --
// A policy fixes the channels that are box-summed per order, the per-pixel
// inputs they need, and how box sums recombine into per-pixel accumulators.

// Forward: channels (C, S, gC, gS), g = f - ref; accumulators (Q, P).
template <typename FT>
struct PolForward {
    static constexpr int NCH = 4, NACC = 2, NAUX = 1;
    template <typename AT>
    __device__ static AT ref(const IO &a, int i, int j)
    {
        return (AT)ld<FT>(a.img, (long)i * a.pitch_in + j);
    }
    template <typename AT>
    __device__ static void load(const IO &a, bool valid, int i, int j, AT ref, AT *aux)
    {
        aux[0] = valid ? (AT)ld<FT>(a.img, (long)i * a.pitch_in + j) - ref : AT(0);
    }
    template <typename AT>
    __device__ static void chans(AT C, AT S, const AT *aux, AT *X)
    {
        X[0] = C;
        X[1] = S;
        X[2] = aux[0] * C;
        X[3] = aux[0] * S;
    }
    template <typename AT>
    __device__ static void recombine(AT v, AT vom, AT C, AT S, const AT *B, const AT *auxc, AT *acc)
    {
        const AT vc = v * C, vs = v * S;
        acc[0] += vc * B[0] + vs * B[1];
        acc[1] += vc * B[2] + vs * B[3];
    }
    template <typename AT>
    __device__ static void finalize(const IO &a, int i, int j, AT ref, const AT *auxc, const AT *acc,
                                    double *red)
    {
        ((FT *)a.out)[(long)i * a.pitch_out + j] = (FT)(ref + acc[1] / acc[0]);
    }
};

// Training forward: channels (C, S, gC, gS, g^2 C, g^2 S); accumulators
// (Q, P, A0, A1, A2) with A_p(z) = sum_{y in B(z)} phi'(g_y - g_z) g_y^p
//   = -sum_m v_m omega_m [C_m(z) Box[g^p S_m] - S_m(z) Box[g^p C_m]],
// phi'(t) = -sum_m v_m omega_m sin(omega_m t).  Outputs u = ref + P/Q and the
// planes Q, E1 = A1 - (u-ref) A0, E2 = A2 - (g_z + u - ref) A1 + g_z (u-ref) A0.
struct PolTrain {
    static constexpr int NCH = 6, NACC = 5, NAUX = 1;
    template <typename AT>
    __device__ static AT ref(const IO &a, int i, int j)
    {
        return (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
    }
    template <typename AT>
    __device__ static void load(const IO &a, bool valid, int i, int j, AT ref, AT *aux)
    {
        aux[0] = valid ? (AT)ld<float>(a.img, (long)i * a.pitch_in + j) - ref : AT(0);
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
        acc[0] += vc * B[0] + vs * B[1];
        acc[1] += vc * B[2] + vs * B[3];
        const AT wc = vom * C, ws = vom * S;
        acc[2] -= wc * B[1] - ws * B[0];
        acc[3] -= wc * B[3] - ws * B[2];
        acc[4] -= wc * B[5] - ws * B[4];
    }
    template <typename AT>
    __device__ static void finalize(const IO &a, int i, int j, AT ref, const AT *auxc, const AT *acc,
                                    double *red)
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

// Backward (adjoint): with alpha = gbar / Q and ut = u - ref, channels
// (alpha C, alpha S, alpha ut C, alpha ut S); one accumulator
//   T1(z) = sum_m v_m { C(z) Box[aC] + S(z) Box[aS]
//           - omega_m [ S(z) (g_z Box[aC] - Box[a ut C]) - C(z) (g_z Box[aS] - Box[a ut S]) ] }
// and dL/df(z) = T1(z) - alpha(z) E1(z); per-workgroup partial sums of
// alpha(x) E2(x) feed dL/dsigma_r.
struct PolBackward {
    static constexpr int NCH = 4, NACC = 1, NAUX = 3;
    template <typename AT>
    __device__ static AT ref(const IO &a, int i, int j)
    {
        return (AT)ld<float>(a.img, (long)i * a.pitch_in + j);
    }
    template <typename AT>
    __device__ static void load(const IO &a, bool valid, int i, int j, AT ref, AT *aux)
    {
        if (valid) {
            const long o = (long)i * a.W + j;
            aux[0] = (AT)ld<float>(a.img, (long)i * a.pitch_in + j) - ref;
            aux[1] = (AT)a.aux0[o] / (AT)a.aux1[o];
            aux[2] = (AT)a.aux2[o] - ref;
        } else {
            aux[0] = aux[1] = aux[2] = AT(0);
        }
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
        const AT gz = auxc[0];
        acc[0] += v * (C * B[0] + S * B[1]) - vom * (S * (gz * B[0] - B[2]) - C * (gz * B[1] - B[3]));
    }
    template <typename AT>
    __device__ static void finalize(const IO &a, int i, int j, AT ref, const AT *auxc, const AT *acc,
                                    double *red)
    {
        const long o = (long)i * a.W + j;
        const AT alpha = auxc[1];
        if (a.out) ((float *)a.out)[o] = (float)(acc[0] - alpha * (AT)a.aux3[o]);
        *red += (double)alpha * (double)a.aux4[o];
    }
};

// ---------------------------------------------------------------- the body --
struct Geom {
    int H, W, pitch_in, pitch_out, rh, rv, S, K;
    double omega_base, delta;
    const double *v;  // folded weights, K entries
    void *ws;         // NACC planes of H*W accumulators, or null when K <= KC
};

template <typename AT, int BLOCK, int KC, class POL, int QUANT, bool KAHAN>
__device__ __forceinline__ void strip_body(const IO &a, const Geom &gm, int bx, int by, AT *lds,
                                           double *red_lds, double *red_out)
{
    constexpr int NCH = POL::NCH;
    constexpr int NACC = POL::NACC;
    constexpr int NAUX = POL::NAUX;
    constexpr int ROWS = NCH * KC;
    constexpr int STRIDE = BLOCK + 1;
    constexpr int NSEG = BLOCK / ROWS;
    static_assert(NSEG >= 1, "too many walker rows for the block");
    AT *Vb = lds;
    AT *Bb = lds + ROWS * STRIDE;

    const int t = threadIdx.x;
    const int H = gm.H, W = gm.W, rh = gm.rh, rv = gm.rv;
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

    // walker assignment (fixed for the whole launch)
    const int wseg = t / ROWS;
    const int wrow = t - wseg * ROWS;
    const int wm = wrow / NCH;
    const int L = (Wt + NSEG - 1) / NSEG;
    const int jlim = min(rh + Wt, rh + (W - j0));   // lane index bound of useful outputs
    const int js = rh + wseg * L;
    const int je = min(jlim, js + L);

    double red = 0.0;

    for (int m0 = 0; m0 < gm.K; m0 += KC) {
        const int kc = min(KC, gm.K - m0);
        const bool first = (m0 == 0);
        const bool last = (m0 + KC >= gm.K);
        const AT om0 = (AT)(gm.omega_base + (double)m0 * gm.delta);
        const AT dlt = (AT)gm.delta;

        AT V[KC][NCH];
        AT Cmp[KAHAN ? KC : 1][NCH];
#pragma unroll
        for (int m = 0; m < KC; ++m)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                V[m][ch] = AT(0);
                Cmp[KAHAN ? m : 0][ch] = AT(0);
            }

        // initial window: rows [i0 - rv, i0 + rv - 1] (the first step adds i0 + rv)
        for (int y = ylo; y < yhi; ++y) {
            AT aux[NAUX];
            POL::template load<AT>(a, colok, y, jx, ref, aux);
            Chain<AT> ch;
            ch.start(colok, aux[0], om0, dlt);
#pragma unroll
            for (int m = 0; m < KC; ++m) {
                if (m < kc) {
                    AT X[NCH];
                    POL::template chans<AT>(quant<QUANT>(ch.c), quant<QUANT>(ch.s), aux, X);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) V[m][c] += X[c];
                    ch.step();
                }
            }
        }

        for (int i = i0; i < i1; ++i) {
            const int yin = i + rv, yout = i - rv - 1;
            const bool vin = colok && (yin < H);
            const bool vout = colok && (yout >= ylo);
            AT auxi[NAUX], auxo[NAUX], auxc[NAUX];
            POL::template load<AT>(a, vin, yin, jx, ref, auxi);
            POL::template load<AT>(a, vout, yout, jx, ref, auxo);
            POL::template load<AT>(a, colok, i, jx, ref, auxc);
            Chain<AT> ci, co, cc;
            ci.start(vin, auxi[0], om0, dlt);
            co.start(vout, auxo[0], om0, dlt);
            cc.start(colok, auxc[0], om0, dlt);
            AT Cc[KC], Sc[KC];

            // ---- phase V: vertical moving sums, transforms by rotation
#pragma unroll
            for (int m = 0; m < KC; ++m) {
                if (m < kc) {
                    AT Xi[NCH], Xo[NCH];
                    POL::template chans<AT>(quant<QUANT>(ci.c), quant<QUANT>(ci.s), auxi, Xi);
                    POL::template chans<AT>(quant<QUANT>(co.c), quant<QUANT>(co.s), auxo, Xo);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        if constexpr (KAHAN) {
                            const AT y = (Xi[c] - Xo[c]) - Cmp[m][c];
                            const AT s = V[m][c] + y;
                            Cmp[m][c] = (s - V[m][c]) - y;
                            V[m][c] = s;
                        } else {
                            V[m][c] += Xi[c] - Xo[c];
                        }
                        Vb[(m * NCH + c) * STRIDE + t] = V[m][c];
                    }
                    Cc[m] = quant<QUANT>(cc.c);
                    Sc[m] = quant<QUANT>(cc.s);
                    ci.step();
                    co.step();
                    cc.step();
                }
            }
            __syncthreads();

            // ---- phase H: horizontal moving sums by sliding walkers
            if (wseg < NSEG && wm < kc && js < je) {
                const AT *vr = Vb + wrow * STRIDE;
                AT *br = Bb + wrow * STRIDE;
                AT acc = AT(0);
                for (int q = js - rh; q <= js + rh; ++q) acc += vr[q];
                br[js] = acc;
                for (int j = js + 1; j < je; ++j) {
                    acc += vr[j + rh] - vr[j - rh - 1];
                    br[j] = acc;
                }
            }
            __syncthreads();

            // ---- phase R: recombination with the shift identity
            if (outlane) {
                AT acc[NACC];
#pragma unroll
                for (int q = 0; q < NACC; ++q) acc[q] = AT(0);
#pragma unroll
                for (int m = 0; m < KC; ++m) {
                    if (m < kc) {
                        AT B[NCH];
#pragma unroll
                        for (int c = 0; c < NCH; ++c) B[c] = Bb[(m * NCH + c) * STRIDE + t];
                        const double om = gm.omega_base + (double)(m0 + m) * gm.delta;
                        const AT v = (AT)gm.v[m0 + m];
                        const AT vom = (AT)(gm.v[m0 + m] * om);
                        POL::template recombine<AT>(v, vom, Cc[m], Sc[m], B, auxc, acc);
                    }
                }
                const long o = (long)i * W + jx;
                if (!first) {
#pragma unroll
                    for (int q = 0; q < NACC; ++q) acc[q] += ((AT *)gm.ws)[q * plane + o];
                }
                if (last) {
                    POL::template finalize<AT>(a, i, jx, ref, auxc, acc, &red);
                } else {
#pragma unroll
                    for (int q = 0; q < NACC; ++q) ((AT *)gm.ws)[q * plane + o] = acc[q];
                }
            }
        }
    }

    if (red_out) {
        // deterministic block reduction (fixed order) of the per-lane sums
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
