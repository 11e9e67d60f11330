// Strip kernel of the bilateral filter with the polynomial range kernel
// (Section 3, p_N, in the scaling of eq. (5)): phi(t) = (1 - t^2 / (2 N sigma_r^2))^N.
//
// A polynomial is shiftable (Section 1), so Algorithm 2 applies with a basis
// of polynomials in the pixel value.  The basis used here is the Chebyshev
// polynomials T_k of the normalised value x = (f - mu) / rho (rho = T / 2,
// mu the midrange of the data the workgroup reads), not the monomials f^k:
// T_k(x) lies in [-1, 1] and the expansion of the kernel in it has
// coefficients bounded by 2 that decay fast enough to be truncated, whereas
// the monomial coefficients of (1 - (x - c)^2 / a^2)^N grow geometrically
// with N (hundreds at N = 37, about 1e7 at N = 82, 1e13 at N = 145) and
// cancel against each other in the sums.  For a centre value c,
//     g_c(x) = phi(rho (x - c)) = sum_k d_k(c) T_k(x)
//     Q(x0) = sum_k d_k(c) Box[T_k](x0)
//     P(x0) = sum_k d_k(c) Box[x T_k](x0),  x T_k = (T_{k+1} + T_{k-1}) / 2,  x T_0 = T_1
//     out = mu + rho P / Q.
// So the stack is one channel per k (T_0 .. T_K), the moving sums are those
// of the raised-cosine kernel (stages V, H and R with the same LDS layout and
// software pipeline, see bsk_device.h), and the per-pixel work that depends on
// c is the coefficient recurrence: the d_k(c) come out of a five-term
// recurrence in k run downwards from d_2N (bsk_plan.cpp), six multiply-adds
// per coefficient.  The channels come from the three-term recurrence
// T_{k+1} = 2 x T_k - T_{k-1}, one multiply-add per value.
#include "bsk_strip.h"

namespace bsk {

// (T_k(x), T_{k+1}(x)) for k = k0, k0 + 2, ...; the start for k0 > 0 by
// doubling, T_{2m} = 2 T_m^2 - 1, T_{2m+1} = 2 T_m T_{m+1} - x,
// T_{2m+2} = 2 T_{m+1}^2 - 1, over the bits of k0.  A pixel outside the image
// starts at zero so all its channels vanish; its value is replaced by 0 first,
// since the stand-in value of an absent pixel may lie far outside [-1, 1],
// where T_k grows without bound.
template <typename AT>
struct ChebPair {
    AT a, b, x2;
    __device__ __forceinline__ void start(bool valid, AT xin, int k0)
    {
        const AT x = valid ? xin : AT(0);
        AT u = AT(1), v = x;
        if (k0 > 0) {
            for (int bit = 31 - __clz(k0); bit >= 0; --bit) {
                const AT t0 = fmat(AT(2) * u, u, AT(-1));
                const AT t1 = fmat(AT(2) * u, v, -x);
                const AT t2 = fmat(AT(2) * v, v, AT(-1));
                const bool one = (k0 >> bit) & 1;
                u = one ? t1 : t0;
                v = one ? t2 : t1;
            }
        }
        const AT z = valid ? AT(1) : AT(0);
        a = z * u;
        b = z * v;
        x2 = AT(2) * x;
    }
    __device__ __forceinline__ void step()
    {
        const AT an = fmat(x2, b, -a);
        const AT bn = fmat(x2, an, -b);
        a = an;
        b = bn;
    }
};

// The coefficient tables are read through ConstPtr (bsk_device.h): scalar
// loads at workgroup-uniform addresses.

// One downward step of the scaled coefficient recurrence, in the variables
// f_j = e_j for even j and f_j = e_j / c for odd j: substituting them removes
// every odd power of c, so with u = c^2
//   even j:  f_j = u (alpha f_{j+1} + gamma f_{j+2} + delta f_{j+3}) + beta f_{j+2} + epsilon f_{j+4}
//   odd j:   f_j = alpha f_{j+1} + (beta + gamma u) f_{j+2} + delta f_{j+3} + epsilon f_{j+4}
// (the row of k = j + 2; w = (f_{j+1}, .., f_{j+4})), six multiply-adds with
// at most one table value each.  Rows above the start shift (epsilon = 1), the
// start row has epsilon = (-1)^N, and the window starts with a single 1 at the
// position that the shifts carry to f_{2N+4}, so every step is the same
// straight-line code.
template <typename AT, bool ODD>
__device__ __forceinline__ AT poly_coef_step(ConstPtr<AT> row, AT u, AT w1, AT w2, AT w3, AT w4)
{
    if constexpr (ODD) {
        AT r = row[1] * w2;
        r = fmat(row[2], u * w2, r);
        r = fmat(row[3], w3, r);
        r = fmat(row[4], w4, r);
        return fmat(row[0], w1, r);
    } else {
        AT t = row[0] * w1;
        t = fmat(row[2], w2, t);
        t = fmat(row[3], w3, t);
        AT r = row[1] * w2;
        r = fmat(row[4], w4, r);
        return fmat(u, t, r);
    }
}

// MULTI: more than one pass (the workspace carries the partial sums and the
// recurrence between passes); a single pass compiles without that code.
// RHC > 0: the horizontal radius as a compile-time constant; the walkers then
// hand box sums to the R stage, as in the strip body.
template <typename AT, int BLOCK, int KR, int KL, bool MULTI, int RHC = 0>
__device__ __forceinline__ void poly_body(const PolyArgs &pa, int bx, int by, AT *lds)
{
    constexpr int ROWS = 2 * KL;
    constexpr int CH = walker_count(BLOCK, ROWS);
    constexpr int G = walker_chunk(BLOCK, CH);
    constexpr int RS = row_stride(BLOCK, CH, G);
    constexpr int BUF = ROWS * RS;
    constexpr int NSUB = KR / KL;
    constexpr int ND = 2 * KR + 2;   // d_{k0-1} .. d_{k0+2KR} of a pass
    constexpr int NWAVE = BLOCK / 64;
    static_assert(KR % KL == 0, "KR must be a multiple of KL");
    static_assert(CH * G >= BLOCK + 1 && RS >= CH * G && ROWS * CH <= BLOCK, "walker geometry");
    static_assert(2 * NWAVE <= kNBuf * BUF, "reduction scratch fits the row buffers");

    const IO &a = pa.io;
    const int t = threadIdx.x;
    const int H = a.H, W = a.W, rh = RHC > 0 ? RHC : pa.rh, rv = pa.rv;
    constexpr bool WBOX = RHC > 0 && sizeof(AT) == 4 && CH == 16 && (2 * RHC + 1) / G + 1 <= 15;
    const int Wt = BLOCK - 2 * rh;
    const int j0 = bx * Wt;
    const int jx = j0 - rh + t;
    const bool colok = (jx >= 0) && (jx < W);
    const int i0 = by * pa.S;
    const int i1 = min(H, i0 + pa.S);
    const int ylo = max(0, i0 - rv);
    const int yhi = min(H, i0 + rv);
    const bool outlane = (t >= rh) && (t < rh + Wt) && colok;
    const long plane = (long)H * W;
    const int jxc = min(max(jx, 0), W - 1);
    auto rowc = [H](int y) { return min(max(y, 0), H - 1); };
    const AT *img = (const AT *)a.img;
    auto fetch = [&](bool valid, int y) {
        const AT x = img[(long)y * a.pitch_in + jxc];
        return valid ? x : AT(0);
    };
    const int wrow = t / CH;
    const int wch = t - wrow * CH;
    constexpr bool ALLWALK = ROWS * CH == BLOCK;
    const bool walker = ALLWALK || wrow < ROWS;
    const int wbase = (wrow >> 1) * (2 * RS) + 2 * (wch * G) + (wrow & 1);
    using V2 = typename Vec2<AT>::type;
    const int phi = t + rh + 1;
    const int plo = t - rh;

    // Midrange of every value this workgroup reads (its columns, rows
    // i0 - rv .. i1 + rv - 1): the normalisation centre mu.
    AT mu;
    {
        AT lo = AT(INFINITY), hi = AT(-INFINITY);
        if (colok) {
            const int ye = min(H, i1 + rv);
            for (int y = ylo; y < ye; ++y) {
                const AT x = img[(long)y * a.pitch_in + jxc];
                lo = fmin(lo, x);
                hi = fmax(hi, x);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off));
            hi = fmax(hi, __shfl_xor(hi, off));
        }
        if ((t & 63) == 0) {
            lds[2 * (t >> 6)] = lo;
            lds[2 * (t >> 6) + 1] = hi;
        }
        __syncthreads();
        lo = lds[0];
        hi = lds[1];
#pragma unroll
        for (int w = 1; w < NWAVE; ++w) {
            lo = fmin(lo, lds[2 * w]);
            hi = fmax(hi, lds[2 * w + 1]);
        }
        __syncthreads();
        mu = AT(0.5) * (lo + hi);
    }
    const AT irho = (AT)pa.inv_rho;
    const AT rho = (AT)pa.rho;
    const ConstPtr<AT> rows = (ConstPtr<AT>)pa.rows;
    const ConstPtr<AT> sig = (ConstPtr<AT>)pa.sig;
    const int n2 = 2 * pa.N;

    // Passes run from the highest channels down: the coefficient recurrence
    // runs downwards too, so a pass continues it from the four values the pass
    // before left in the workspace (planes 2 .. 5) instead of from d_2N.
    AT *const ws = (AT *)pa.ws;
    for (int p0 = MULTI ? pa.NP - KR : 0; p0 >= 0; p0 -= KR) {
        const int k0 = 2 * p0;   // first channel of the pass
        const bool top_pass = !MULTI || (p0 + KR >= pa.NP);   // first to run
        const bool base = !MULTI || (p0 == 0);                 // last to run: channels 0 and 1

        AT V[KR][2];
#pragma unroll
        for (int m = 0; m < KR; ++m) V[m][0] = V[m][1] = AT(0);

        // initial window: rows [i0 - rv, i0 + rv - 1] (the first step adds i0 + rv)
        {
            AT raw = fetch(colok, rowc(ylo));
            for (int y = ylo; y < yhi; ++y) {
                const AT x = (raw - mu) * irho;
                raw = fetch(colok, rowc(y + 1));
                ChebPair<AT> ch;
                ch.start(colok, x, k0);
#pragma unroll
                for (int m = 0; m < KR; ++m) {
                    V[m][0] += ch.a;
                    V[m][1] += ch.b;
                    ch.step();
                }
            }
        }

        AT rin, rout, rc;
        {
            const int yin = i0 + rv, yout = i0 - rv - 1;
            rin = fetch(colok && yin < H, rowc(yin));
            rout = fetch(colok && yout >= ylo, rowc(yout));
            rc = fetch(colok, i0);
        }
        ChebPair<AT> ci, co;
        ci.a = ci.b = ci.x2 = co.a = co.b = co.x2 = AT(0);
        AT dd[ND];
#pragma unroll
        for (int q = 0; q < ND; ++q) dd[q] = AT(0);
        AT accQ = AT(0), accP = AT(0);   // Q and 2P of the row in the R stage
        AT wsQ = AT(0), wsP = AT(0);     // the pass above's Q and 2P, read when the row starts
        int bv = 0;

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
                if (!(actV || actH || actR)) continue;
                const int bH = bv == 0 ? kNBuf - 1 : bv - 1;
                const int bR = bH == 0 ? kNBuf - 1 : bH - 1;
                V2 *const VbV = reinterpret_cast<V2 *>(lds + bv * BUF);
                AT *const VbH = lds + bH * BUF;
                const V2 *const VbR = reinterpret_cast<const V2 *>(lds + bR * BUF);

                // wave priorities per stage, as in the strip body (H above R above V)
                __builtin_amdgcn_s_setprio(1);
                // ---- R stage: coefficients of the centre value (first sub-phase),
                //      then the box sums of the pass's channels
                if (actR && outlane) {
                    if (sR == 0) {
                        const AT c = (rc - mu) * irho;
                        const AT u = c * c;
                        rc = fetch(colok, rowc(iR + 1));
                        // f_j for j from 2N down to k0 - 1; values above the
                        // register range only feed the recurrence
                        const long o = (long)iR * W + jx;
                        const int jtop = k0 + 2 * KR;   // even, as are k0 and 2N
                        AT w1, w2, w3, w4;
                        if (top_pass) {
                            // the window above the first step j1 = max(2N, jtop):
                            // a single 1 where the shifts carry it to f_{2N+4}
                            const int j1 = max(n2, jtop);
                            w1 = ((j1 + 1 - n2) & 3) == 0 ? AT(1) : AT(0);
                            w2 = ((j1 + 2 - n2) & 3) == 0 ? AT(1) : AT(0);
                            w3 = ((j1 + 3 - n2) & 3) == 0 ? AT(1) : AT(0);
                            w4 = ((j1 + 4 - n2) & 3) == 0 ? AT(1) : AT(0);
                            // steps j, j - 1, ... down to jtop + 1, four at a time (the
                            // window then rotates by renaming alone), after one pair of
                            // steps when their count is not a multiple of four
                            int j = n2;
                            if (n2 > jtop && ((n2 - jtop) & 2)) {
                                const AT fe = poly_coef_step<AT, false>(rows + (long)kPolyRow * (j + 2), u, w1, w2, w3, w4);
                                const AT fo = poly_coef_step<AT, true>(rows + (long)kPolyRow * (j + 1), u, fe, w1, w2, w3);
                                w4 = w2;
                                w3 = w1;
                                w2 = fe;
                                w1 = fo;
                                j -= 2;
                            }
                            for (; j > jtop; j -= 4) {
                                const ConstPtr<AT> r0 = rows + (long)kPolyRow * (j - 1);   // row of j - 3
                                const AT fa = poly_coef_step<AT, false>(r0 + 3 * kPolyRow, u, w1, w2, w3, w4);
                                const AT fb = poly_coef_step<AT, true>(r0 + 2 * kPolyRow, u, fa, w1, w2, w3);
                                const AT fc = poly_coef_step<AT, false>(r0 + kPolyRow, u, fb, fa, w1, w2);
                                const AT fd = poly_coef_step<AT, true>(r0, u, fc, fb, fa, w1);
                                w4 = fa;
                                w3 = fb;
                                w2 = fc;
                                w1 = fd;
                            }
                        } else {
                            // Q and 2P so far (added when the row ends) and f_{jtop+1} ..
                            // f_{jtop+4}, from the pass above
                            wsQ = ws[o];
                            wsP = ws[plane + o];
                            w1 = ws[2 * plane + o];
                            w2 = ws[3 * plane + o];
                            w3 = ws[4 * plane + o];
                            w4 = ws[5 * plane + o];
                        }
                        const ConstPtr<AT> rp = rows + (long)kPolyRow * (k0 + 1);   // row of j = k0 - 1
#pragma unroll
                        for (int q = ND - 1; q >= 0; --q) {
                            // j = k0 - 1 + q is odd exactly when q is even
                            const AT e = (q & 1) ? poly_coef_step<AT, false>(rp + kPolyRow * q, u, w1, w2, w3, w4)
                                                 : poly_coef_step<AT, true>(rp + kPolyRow * q, u, w1, w2, w3, w4);
                            dd[q] = e;
                            w4 = w3;
                            w3 = w2;
                            w2 = w1;
                            w1 = e;
                        }
                        if (!base) {
                            // f_{k0+1} .. f_{k0+4} for the pass below
                            ws[2 * plane + o] = dd[2];
                            ws[3 * plane + o] = dd[3];
                            ws[4 * plane + o] = dd[4];
                            ws[5 * plane + o] = dd[5];
                        }
                        // d_k = s_k e_k = s_k f_k (even k), s_k c f_k (odd k); s_k = 0
                        // past the kept coefficients and for k = -1
                        const ConstPtr<AT> sp = sig + k0;
#pragma unroll
                        for (int q = 0; q < ND; ++q) dd[q] *= (q & 1) ? sp[q] : sp[q] * c;
                        accQ = accP = AT(0);
                    }
#pragma unroll
                    for (int k = 0; k < KL; ++k) {
                        const int m = sR * KL + k;
                        const V2 *prow = VbR + k * RS;
                        AT Ba, Bb;   // Box[T_{k0+2m}], Box[T_{k0+2m+1}]
                        if constexpr (WBOX) {
                            const V2 bx2 = prow[phi];
                            Ba = bx2.x;
                            Bb = bx2.y;
                        } else {
                            const V2 hi = prow[phi], lo = prow[plo];
                            Ba = hi.x - lo.x;
                            Bb = hi.y - lo.y;
                        }
                        accQ = fmat(dd[2 * m + 1], Ba, fmat(dd[2 * m + 2], Bb, accQ));
                        accP = fmat(dd[2 * m] + dd[2 * m + 2], Ba, fmat(dd[2 * m + 1] + dd[2 * m + 3], Bb, accP));
                        // x T_0 = T_1 carries d_0 in full: 2P gains another d_0 Box[T_1]
                        if (m == 0 && base) accP = fmat(dd[1], Bb, accP);
                    }
                }

                __builtin_amdgcn_s_setprio(2);
                // ---- H stage: every row of buffer t - 1 into its exclusive prefix sums, in place
                if (actH) {
                    AT loc[G];
                    AT run = AT(0);
                    if (walker) {
#pragma unroll
                        for (int u = 0; u < G; ++u) loc[u] = VbH[wbase + 2 * u];
#pragma unroll
                        for (int u = 0; u < G; ++u) {
                            const AT x = loc[u];
                            loc[u] = run;
                            run += x;
                        }
                    }
                    const AT off = group_exclusive_scan<CH>(run, wch);
                    if (walker) {
                        if constexpr (WBOX) {
                            // box sums: E(p) - E(p - 2 rh - 1), the second a fixed DPP
                            // shift and element away (strip_body has the derivation)
                            constexpr int D = 2 * RHC + 1, QS = D / G, DR = D % G;
                            AT E[G];
#pragma unroll
                            for (int u = 0; u < G; ++u) E[u] = loc[u] + off;
#pragma unroll
                            for (int u = 0; u < G; ++u) {
                                const AT lo = u >= DR ? dpp_row_shr<QS>(E[u >= DR ? u - DR : 0])
                                                      : dpp_row_shr<QS + 1>(E[u < DR ? u - DR + G : 0]);
                                VbH[wbase + 2 * u] = E[u] - lo;
                            }
                        } else {
#pragma unroll
                            for (int u = 0; u < G; ++u) VbH[wbase + 2 * u] = loc[u] + off;
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
                        ci.start(vin, (rin - mu) * irho, k0);
                        co.start(vout, (rout - mu) * irho, k0);
                        rin = fetch(colok && yin + 1 < H, rowc(yin + 1));
                        rout = fetch(colok && yout + 1 >= ylo, rowc(yout + 1));
                    }
#pragma unroll
                    for (int k = 0; k < KL; ++k) {
                        const int m = h * KL + k;
                        V[m][0] = (V[m][0] + ci.a) - co.a;
                        V[m][1] = (V[m][1] + ci.b) - co.b;
                        VbV[k * RS + t] = Vec2<AT>::make(V[m][0], V[m][1]);
                        ci.step();
                        co.step();
                    }
                }

                // ---- row iR complete: continue or finish its accumulators
                if (actR && sR == NSUB - 1 && outlane) {
                    const long o = (long)iR * W + jx;
                    if (!top_pass) {
                        accQ += wsQ;
                        accP += wsP;
                    }
                    if (base) {
                        ((AT *)a.out)[(long)iR * a.pitch_out + jx] = mu + rho * (AT(0.5) * accP / accQ);
                    } else {
                        ws[o] = accQ;
                        ws[plane + o] = accP;
                    }
                }
                __syncthreads();
                bv = bv == kNBuf - 1 ? 0 : bv + 1;
            }
        }
    }
}

// Pass shapes: KR channel pairs in registers per pass, KL pairs per pipeline
// interval (2 KL LDS rows per buffer).  The three row buffers of the 256-lane
// FP32 kernel take 52 KiB, so three workgroups share a compute unit.
constexpr int kr_poly_f32(int block) { return block == 1024 ? 8 : 16; }
constexpr int kl_poly_f32(int block) { return block == 256 ? 8 : block == 512 ? 4 : 2; }
constexpr int kr_poly_f64(int block) { return block == 256 ? 8 : block == 512 ? 4 : 2; }
constexpr int kl_poly_f64(int block) { return block == 1024 ? 1 : 2; }
constexpr int poly_lds_occupancy(int bytes) { return bytes <= 160 * 1024 / 3 ? 3 : bytes <= 80 * 1024 ? 2 : 1; }
template <typename AT, int BLOCK, int KL>
constexpr int poly_minb()
{
    return BLOCK == 1024 ? 1 : (poly_lds_occupancy(strip_lds_elems<2, KL, BLOCK>() * (int)sizeof(AT)) >= 3 ? 3 : 2);
}

template <typename AT, int BLOCK, int KR, int KL, bool MULTI, int RHC = 0>
__global__ void __launch_bounds__(BLOCK, (poly_minb<AT, BLOCK, KL>())) poly_kernel(const PolyArgs a)
{
    __shared__ __align__(16) AT lds[strip_lds_elems<2, KL, BLOCK>()];
    int bx, by;
    if (!xcd_tile((a.io.W + BLOCK - 2 * a.rh - 1) / (BLOCK - 2 * a.rh), (a.io.H + a.S - 1) / a.S, &bx, &by)) return;
    poly_body<AT, BLOCK, KR, KL, MULTI, RHC>(a, bx, by, lds);
}

template <typename AT, int BLOCK, int KR, int KL, int RHC = 0>
static hipError_t poly_launch(const PolyArgs &a, hipStream_t s, int *occ)
{
    if (occ) return query_occupancy((const void *)poly_kernel<AT, BLOCK, KR, KL, true, RHC>, BLOCK, occ);
    if (RHC > 0 && a.rh != RHC) return hipErrorInvalidValue;
    const int Wt = BLOCK - 2 * a.rh;
    if (Wt < 1 || a.S < 1 || a.NP < KR || a.NP % KR != 0) return hipErrorInvalidValue;
    const bool multi = a.NP > KR;
    if (multi && !a.ws) return hipErrorInvalidValue;
    const dim3 grid(xcd_grid((a.io.W + Wt - 1) / Wt, (a.io.H + a.S - 1) / a.S));
    if (multi) hipLaunchKernelGGL((poly_kernel<AT, BLOCK, KR, KL, true, RHC>), grid, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((poly_kernel<AT, BLOCK, KR, KL, false, RHC>), grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// 256 lanes at the radii of the compile-time-radius strip kernels: walkers
// that hand out box sums
template <int KR, int KL>
static hipError_t poly32_radius(const PolyArgs &a, hipStream_t s, int *occ)
{
    switch (a.rh) {
    case 3: return poly_launch<float, 256, KR, KL, 3>(a, s, occ);
    case 5: return poly_launch<float, 256, KR, KL, 5>(a, s, occ);
    case 8: return poly_launch<float, 256, KR, KL, 8>(a, s, occ);
    case 10: return poly_launch<float, 256, KR, KL, 10>(a, s, occ);
    case 16: return poly_launch<float, 256, KR, KL, 16>(a, s, occ);
    case 20: return poly_launch<float, 256, KR, KL, 20>(a, s, occ);
    case 25: return poly_launch<float, 256, KR, KL, 25>(a, s, occ);
    case 32: return poly_launch<float, 256, KR, KL, 32>(a, s, occ);
    default: return poly_launch<float, 256, KR, KL>(a, s, occ);
    }
}

// The 24-pair pass of 256 lanes, at those radii only: 158 VGPRs and three
// workgroups per CU (the run-time-radius kernel of that size spills), so many
// channel pairs take fewer passes.
constexpr int kbig_poly_f32 = 24;
bool big_chunk_poly_ok(int block, int rh)
{
    switch (rh) {
    case 3: case 5: case 8: case 10: case 16: case 20: case 25: case 32: return block == 256;
    default: return false;
    }
}
static hipError_t poly32_big(const PolyArgs &a, hipStream_t s, int *occ)
{
    constexpr int KR = kbig_poly_f32, KL = kl_poly_f32(256);
    switch (a.rh) {
    case 3: return poly_launch<float, 256, KR, KL, 3>(a, s, occ);
    case 5: return poly_launch<float, 256, KR, KL, 5>(a, s, occ);
    case 8: return poly_launch<float, 256, KR, KL, 8>(a, s, occ);
    case 10: return poly_launch<float, 256, KR, KL, 10>(a, s, occ);
    case 16: return poly_launch<float, 256, KR, KL, 16>(a, s, occ);
    case 20: return poly_launch<float, 256, KR, KL, 20>(a, s, occ);
    case 25: return poly_launch<float, 256, KR, KL, 25>(a, s, occ);
    case 32: return poly_launch<float, 256, KR, KL, 32>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}

template <int BLOCK>
static hipError_t poly32_block(const PolyArgs &a, int kc, hipStream_t s, int *occ)
{
    constexpr int KR = kr_poly_f32(BLOCK), KL = kl_poly_f32(BLOCK);
    constexpr int KLH = KL < KR / 2 ? KL : KR / 2;
    if constexpr (BLOCK == 256) {
        if (kc == kbig_poly_f32) return poly32_big(a, s, occ);
        if (kc == KR) return poly32_radius<KR, KL>(a, s, occ);
        if (kc == KR / 2) return poly32_radius<KR / 2, KLH>(a, s, occ);
    }
    if (kc == KR) return poly_launch<float, BLOCK, KR, KL>(a, s, occ);
    if (kc == KR / 2) return poly_launch<float, BLOCK, KR / 2, KLH>(a, s, occ);
    return hipErrorInvalidValue;
}

int chunk_poly_f32(int block) { return block == 1024 ? kr_poly_f32(1024) : kr_poly_f32(256); }
int big_chunk_poly_f32(int block, int rh) { return big_chunk_poly_ok(block, rh) ? kbig_poly_f32 : 0; }
int chunk_poly_f64(int block)
{
    return block == 256 ? kr_poly_f64(256) : block == 512 ? kr_poly_f64(512) : kr_poly_f64(1024);
}

hipError_t launch_poly_f32(const PolyArgs &a, int block, int kc, hipStream_t s, int *occ)
{
    switch (block) {
    case 256: return poly32_block<256>(a, kc, s, occ);
    case 512: return poly32_block<512>(a, kc, s, occ);
    case 1024: return poly32_block<1024>(a, kc, s, occ);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_poly_f64(const PolyArgs &a, int block, hipStream_t s, int *occ)
{
    switch (block) {
    case 256: return poly_launch<double, 256, kr_poly_f64(256), kl_poly_f64(256)>(a, s, occ);
    case 512: return poly_launch<double, 512, kr_poly_f64(512), kl_poly_f64(512)>(a, s, occ);
    case 1024: return poly_launch<double, 1024, kr_poly_f64(1024), kl_poly_f64(1024)>(a, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bsk
