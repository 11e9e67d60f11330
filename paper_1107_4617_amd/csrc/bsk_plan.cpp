// Host-side plan of the shiftable range kernel: order selection, folded
// frequencies and FP64 binomial weights, truncation.
//
// Section 3 gives q_N(t) = cos^N(pi t / 2T) on [-T, T], of shiftability order
// N+1; Theorem 3.3, eq. (6), rescales it as q_N(t / sqrt N) -> Gaussian.  With
// gamma = 1 / sigma_r the kernel is phi(t) = cos^N(gamma t / sqrt N), and the
// binomial theorem on cos a = (e^{ia} + e^{-ia}) / 2 gives
//     phi(t) = sum_{n=0..N} w_n cos((2n - N) gamma t / sqrt N),  w_n = 2^-N C(N, n),
// a finite sum of exponentials (Section 1), hence shiftable.
#include <cmath>

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

}  // namespace bsk
