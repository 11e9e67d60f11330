// Host-side plan of the shiftable range kernel: order selection, folded
// frequencies and FP64 binomial weights, truncation.
//
// Section 3 gives q_N(t) = cos^N(pi t / 2T) on [-T, T], of shiftability order
// N+1; Theorem 3.3, eq. (6), rescales it as q_N(t / sqrt N) -> Gaussian.  With
// gamma = 1 / sigma_r the kernel is phi(t) = cos^N(gamma t / sqrt N), and the
// binomial theorem on cos a = (e^{ia} + e^{-ia}) / 2 gives
//     phi(t) = sum_{n=0..N} w_n cos((2n - N) gamma t / sqrt N),  w_n = 2^-N C(N, n),
// a finite sum of exponentials (Section 1), hence shiftable.
#include <algorithm>
#include <cmath>
#include <limits>

#include "bsk_internal.h"

namespace bsk {

int order_for(double sigma_r, double T)
{
    // Smallest N with gamma T / sqrt N <= pi / 2: the kernel is then
    // non-negative and unimodal on [-T, T] (Section 3.1, N_0 = O(T^2/sigma^2)).
    const double x = 2.0 * T / (M_PI * sigma_r);
    return (int)std::ceil(x * x);
}

// w_h = 2^-N C(N, h) for h = floor(N / 2), as a product of factors
// (N - h + i) / (4 i) that each lie in (1/4, 1], so nothing under- or
// overflows before the end.
static double central_weight(int N)
{
    const int h = N / 2;
    double w = 1.0;
    for (int i = 1; i <= h; ++i) w *= (double)(N - h + i) / (4.0 * (double)i);
    if (N & 1) w *= 0.5;
    return w;
}

void plan_counts(int N, double eps, int *K, double *dropped)
{
    if (N == 0) {
        if (K) *K = 1;
        if (dropped) *dropped = 0.0;
        return;
    }
    const int h = N / 2;
    const int full = (N & 1) ? (N + 1) / 2 : N / 2 + 1;
    // unfolded weights from the centre outwards: w_{n-1} = w_n n / (N - n + 1);
    // they decrease, so once one falls below eps every later one does too
    double w = central_weight(N), drop = 0.0;
    int k = 0;
    bool stop = false;
    for (int m = 0; m < full; ++m) {
        const int n = h - m;
        const double mult = ((N & 1) == 0 && m == 0) ? 1.0 : 2.0;
        if (eps > 0.0 && w < eps) stop = true;
        if (stop) drop += mult * w;
        else ++k;
        w = w * (double)n / (double)(N - n + 1);
    }
    if (K) *K = k;
    if (dropped) *dropped = drop;
}

int make_plan(int N, double sigma_r, double eps, Plan *p)
{
    p->N = N;
    p->gamma = 1.0 / sigma_r;
    p->dropped = 0.0;
    if (N == 0) {
        // phi = 1: the box mean (N = 0 is allowed in Section 3).
        p->K = p->K_full = 1;
        p->omega_base = 0.0;
        p->delta = 0.0;
        p->v[0] = 1.0;
        p->start_mode = 0;
        return 0;
    }
    const double s = p->gamma / std::sqrt((double)N);   // frequency unit
    const int h = N / 2;
    const int full = (N & 1) ? (N + 1) / 2 : N / 2 + 1;
    p->K_full = full;
    // Folded order m pairs n = h - m with N - n: frequency |2n - N| s.
    //   N even: m = 0 is the zero frequency (n = N/2, single weight), then 2 m s.
    //   N odd:  (2m + 1) s.
    p->omega_base = (N & 1) ? s : 0.0;
    p->delta = 2.0 * s;
    p->start_mode = (N & 1) ? 1 : 0;
    double w = central_weight(N);
    int k = 0;
    bool stop = false;
    for (int m = 0; m < full; ++m) {
        const int n = h - m;
        const double mult = ((N & 1) == 0 && m == 0) ? 1.0 : 2.0;
        if (eps > 0.0 && w < eps) stop = true;   // weights decrease outwards
        if (stop) {
            p->dropped += mult * w;
        } else {
            if (k >= kMaxOrders) return -2;
            p->v[k++] = mult * w;
        }
        w = w * (double)n / (double)(N - n + 1);
    }
    p->K = k;
    return 0;
}

int make_spatial_plan(int Ns, double sigma_s, SpatialPlan *sp)
{
    if (Ns < 0 || Ns > 2 * kMaxSpatialFreq || !(sigma_s > 0.0) || !std::isfinite(sigma_s)) return -1;
    *sp = SpatialPlan();
    sp->Ns = Ns;
    sp->sigma = sigma_s;
    if (Ns == 0) return 0;   // the box
    // 2^-Ns C(Ns, j), exact for Ns <= 6
    double c = 1.0;
    double binom[2 * kMaxSpatialFreq + 1];
    for (int j = 0; j <= Ns; ++j) {
        binom[j] = c;
        c = c * (double)(Ns - j) / (double)(j + 1);
    }
    const double scale = std::ldexp(1.0, -Ns);
    const double unit = 1.0 / (sigma_s * std::sqrt((double)Ns));
    sp->nsc = (Ns + 1) / 2;
    sp->even = (Ns % 2) == 0;
    sp->u0 = sp->even ? binom[Ns / 2] * scale : 0.0;
    for (int j = 0; j < sp->nsc; ++j) {
        sp->u[j] = 2.0 * binom[j] * scale;
        sp->nu[j] = (double)(Ns - 2 * j) * unit;
    }
    return 0;
}

// ------------------------------------------------ polynomial range kernel --
//
// Section 3 gives p_N(t) = (1 - t^2/T^2)^N on [-T, T], of shiftability order
// 2N + 1; eq. (5) rescales it as p_N(t / sqrt N) -> exp(-t^2 / T^2).  With
// the bound of p_N set to sqrt(2) sigma_r the kernel is
// phi(t) = (1 - t^2 / (2 N sigma_r^2))^N, tending to exp(-t^2 / 2 sigma_r^2).

int poly_order_for(double sigma_r, double T)
{
    const double x = T / sigma_r;
    return (int)std::ceil(0.5 * x * x);
}

// Chebyshev coefficients of g_c(x) = h(x)^N, h(x) = 1 - (x - c)^2 / a^2.
// Writing g' in the second-kind basis (T_k' = k U_{k-1}), multiplying by x as
// x U_j = (U_{j+1} + U_{j-1}) / 2 and T_k = (U_k - U_{k-2}) / 2, the equation
// (a^2 - (x - c)^2) g' + 2 N (x - c) g = 0 becomes, coefficient by coefficient,
//   (2N - k + 2) d_{k-2} + 4c (k - 1 - N) d_{k-1} + (4 A - 2) k d_k
//       + 4c (k + 1 + N) d_{k+1} - (2N + k + 2) d_{k+2} = 0,   A = a^2 - c^2,
// for k >= 3; for k = 2 the first factor is 4N (T_0 = U_0 carries a full
// coefficient).  The leading coefficient is d_2N = (-1/a^2)^N 2^(1-2N), the
// same for every c.  Run downwards from it, the recurrence is stable in the
// relative sense: rounding errors grow no faster than the coefficients.
static double poly_step(int N, double A, double c, int k, const double *d /* d_{k-1}, d_k, d_{k+1}, d_{k+2} */)
{
    const double den = k >= 3 ? (double)(2 * N - k + 2) : 4.0 * N;
    const double num = 4.0 * c * (double)(k - 1 - N) * d[0] + (4.0 * A - 2.0) * (double)k * d[1]
                     + 4.0 * c * (double)(k + 1 + N) * d[2] - (double)(2 * N + k + 2) * d[3];
    return -num / den;
}

int make_poly_plan(int N, double sigma_r, double T, double eps, PolyPlan *pp)
{
    if (N < 0 || N > kMaxPolyOrder || !(sigma_r > 0.0) || !(T > 0.0) || !std::isfinite(sigma_r) ||
        !std::isfinite(T))
        return -1;
    PolyPlan &p = *pp;
    p.N = N;
    p.rho = 0.5 * T;
    p.ahat = N > 0 ? std::sqrt(2.0 * N) * sigma_r / p.rho : 0.0;
    p.top = (N & 1) ? -1.0 : 1.0;
    const int n2 = 2 * N;
    p.lsig.assign(n2 + 1, -std::numeric_limits<double>::infinity());
    p.rows.assign((size_t)(n2 + 3) * kPolyRow, 0.0);
    // the step that yields e_2N takes it from a 1 four places up: e_2N = top
    // (the device shifts that 1 down with rows whose only entry is epsilon = 1)
    p.rows[(size_t)(n2 + 2) * kPolyRow + 4] = p.top;
    if (N == 0) {
        // g = 1: d_0 = 1 and nothing to recur
        p.lsig[0] = 0.0;
        p.K = 1;
        p.bound = 0.0;
        return 0;
    }
    // Scale profile: ln max_c |d_k(c)| over a grid of centres, each run of the
    // recurrence in FP64 from d_2N = 1 with the true magnitude tracked apart.
    const double a2 = p.ahat * p.ahat;
    const double ltop = -(double)N * std::log(a2) - (double)(n2 - 1) * std::log(2.0);
    const int grid = 257;
    std::vector<double> lg(n2 + 1);
    for (int gi = 0; gi < grid; ++gi) {
        const double c = -1.0 + 2.0 * gi / (grid - 1);
        const double A = a2 - c * c;
        double w[4] = {1.0, 0.0, 0.0, 0.0};   // d_{j+1} .. d_{j+4}, starting above d_2N - 1
        double shift = 0.0;
        lg[n2] = ltop;
        for (int j = n2 - 1; j >= 0; --j) {
            double dj = poly_step(N, A, c, j + 2, w);
            if (std::fabs(dj) > 1e150) {
                dj *= 1e-150;
                for (double &x : w) x *= 1e-150;
                shift += 150.0 * std::log(10.0);
            }
            lg[j] = dj != 0.0 ? std::log(std::fabs(dj)) + shift + ltop : -std::numeric_limits<double>::infinity();
            w[3] = w[2];
            w[2] = w[1];
            w[1] = w[0];
            w[0] = dj;
        }
        for (int k = 0; k <= n2; ++k) p.lsig[k] = std::max(p.lsig[k], lg[k]);
    }
    for (int k = 0; k <= n2; ++k)
        if (!std::isfinite(p.lsig[k])) p.lsig[k] = -700.0;   // never the largest anywhere: negligible
    // Truncation: keep d_k for k < K, the smallest K whose dropped tail has
    // sum_k max_c |d_k(c)| <= eps (the kernel's peak g_c(c) is 1).
    p.K = n2 + 1;
    p.bound = 0.0;
    if (eps > 0.0) {
        double tail = 0.0;
        int K = n2 + 1;
        for (int k = n2; k >= 1; --k) {
            const double t = tail + std::exp(p.lsig[k]);
            if (t > eps) break;
            tail = t;
            K = k;
        }
        p.K = K;
        p.bound = tail;
    }
    // Scaled step coefficients: d_k = s_k e_k with s_k = exp(lsig[k]).
    auto ratio = [&](int j, int k) { return j > n2 ? 0.0 : std::exp(p.lsig[j] - p.lsig[k]); };
    for (int k = 2; k <= n2 + 1; ++k) {
        const double den = k >= 3 ? (double)(n2 - k + 2) : 4.0 * N;
        double *row = &p.rows[(size_t)k * kPolyRow];
        row[0] = -4.0 * (double)(k - 1 - N) * ratio(k - 1, k - 2) / den;       // alpha (times c e_{k-1})
        row[1] = -(4.0 * a2 - 2.0) * (double)k * ratio(k, k - 2) / den;         // beta (times e_k)
        row[2] = 4.0 * (double)k * ratio(k, k - 2) / den;                       // gamma (times c^2 e_k)
        row[3] = -4.0 * (double)(k + 1 + N) * ratio(k + 1, k - 2) / den;        // delta (times c e_{k+1})
        row[4] = (double)(n2 + k + 2) * ratio(k + 2, k - 2) / den;              // epsilon (times e_{k+2})
    }
    return 0;
}

}  // namespace bsk
