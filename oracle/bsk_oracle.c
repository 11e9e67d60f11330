/*
 * FP64 CPU oracle for the constant-time bilateral filter of
 * K. N. Chaudhury, "Constant-time filtering using shiftable kernels".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it, and it shares no code, header, table or
 * constant with the HIP sources.
 *
 * What it computes (Section 2, eq. (3)): for every pixel x,
 *     P(x) = sum_{y in B(x)} phi(f(y) - f(x)) f(y)
 *     Q(x) = sum_{y in B(x)} phi(f(y) - f(x))          (the normaliser eta(x))
 *     out(x) = P(x) / Q(x)
 * with
 *   - a box spatial kernel: B(x) is the (2r+1)x(2r+1) square centred at x,
 *     truncated at the image border (pixels outside the image are absent).
 *     The box is the degree-0 member of the separable family of Section 3
 *     (N = 0 is allowed there), so the spatial basis has a single function;
 *   - the raised-cosine range kernel q_N of Section 3 in the rescaled form of
 *     Theorem 3.3, eq. (6): phi(t) = [cos(t / (sigma_r sqrt(N)))]^N, which
 *     tends to exp(-t^2 / (2 sigma_r^2)) as N grows.  Matching eq. (6) with
 *     gamma = pi/(2T) gives gamma = 1/sigma_r for a target Gaussian of
 *     standard deviation sigma_r.  N = 0 gives phi = 1 (the box mean).
 *
 * Algorithm 2 reaches this result exactly (up to rounding) because the
 * raised cosine is a finite sum of exponentials (Section 1), so the oracle is
 * the definition itself, evaluated window element by window element, with
 * no expansion, no moving sums and no folding.
 *
 * The truncated variant evaluates, directly, the kernel that remains after
 * the less significant basis functions are discarded (Section 3.1, last
 * paragraph): phi_eps(t) = sum_{n : w_n >= eps} w_n cos(omega_n t) with
 * w_n = 2^-N C(N, n) and omega_n = (2n - N) / (sigma_r sqrt(N)).
 *
 * The gradient routine differentiates the same definition by hand (chain
 * rule through P, Q and the kernel), again by direct window sums.
 *
 * The *_sp functions add the separable raised-cosine spatial kernel of
 * Algorithms 1 and 2 with M > 1 (defined with oracle_spatial_weight below).
 *
 * The *_nlm2 functions compute the two-pixel-patch form of the non-local
 * means filter of the Discussion (Section 5): the range kernel compares the
 * patches {y, y + u} and {x, x + u} through the separable product of two
 * raised cosines, one per patch pixel (the shiftable approximation of the
 * anisotropic Gaussian phi(t_1, .., t_p) with p = 2).
 *
 * The *_poly functions use instead the polynomial range kernel p_N of
 * Section 3 in the scaling of the Gaussian-approximation theorem, eq. (5):
 * p_N(t / sqrt N) with the bound T of p_N set to sqrt(2) sigma_r, i.e.
 * phi(t) = (1 - t^2 / (2 N sigma_r^2))^N, which tends to
 * exp(-t^2 / (2 sigma_r^2)).  A polynomial is shiftable (Section 1), so the
 * method again reaches the definition exactly and the oracle is the
 * definition, evaluated directly (no expansion).
 *
 * Conventions: images are row-major, H rows by W columns; float inputs are
 * widened exactly to double; accumulation is sequential in row-major window
 * order; rows are distributed over OpenMP threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Smallest order N for which the rescaled argument t/(sigma_r sqrt N) stays
 * within [-pi/2, pi/2] for |t| <= T, i.e. the kernel stays non-negative and
 * unimodal on [-T, T]; this is the threshold N_0 = O(T^2/sigma^2) of
 * Section 3.1. */
int oracle_order_for(double sigma_r, double T)
{
    double x = 2.0 * T / (M_PI * sigma_r);
    return (int)ceil(x * x);
}

/* c^N by repeated squaring; the sign of c is kept, so odd N and negative
 * cosines are handled. */
static double ipow(double c, int N)
{
    double acc = 1.0, b = c;
    unsigned n = (unsigned)N;
    while (n) {
        if (n & 1u) acc *= b;
        b *= b;
        n >>= 1;
    }
    return acc;
}

/* Range kernel phi(t) = cos^N(t / (sigma_r sqrt N)); Section 3, q_N, in the
 * scaling of eq. (6). */
double oracle_kernel(double t, double sigma_r, int N)
{
    if (N == 0) return 1.0;
    double a = t / (sigma_r * sqrt((double)N));
    return ipow(cos(a), N);
}

/* d phi / d t. */
double oracle_kernel_deriv(double t, double sigma_r, int N)
{
    if (N == 0) return 0.0;
    double s = sigma_r * sqrt((double)N);
    double a = t / s;
    return -(double)N * ipow(cos(a), N - 1) * sin(a) / s;
}

/* Binomial weights w_n = 2^-N C(N, n), n = 0..N, into w[0..N].
 * Section 3.1 discards the basis functions whose weight falls below a
 * threshold, so deciding w_n < eps at an eps equal to a kept weight needs each
 * weight as the double nearest its exact value.  For N <= 130 the binomial
 * coefficients come from Pascal's triangle in unsigned 128-bit integers
 * (C(130, 65) < 2^127, so every entry is exact); the conversion to double
 * rounds once to nearest and the scaling by 2^-N is exact.  Beyond N = 130 the
 * log-gamma form is used, which is accurate to about 1e-13 relative. */
#define ORACLE_EXACT_BINOM_MAX 130
static void binom_row(int N, double *w)
{
    if (N <= ORACLE_EXACT_BINOM_MAX) {
        unsigned __int128 c[ORACLE_EXACT_BINOM_MAX + 1];
        c[0] = 1;
        for (int row = 1; row <= N; ++row) {
            c[row] = 1;
            for (int n = row - 1; n >= 1; --n) c[n] += c[n - 1];
        }
        for (int n = 0; n <= N; ++n) w[n] = ldexp((double)c[n], -N);
        return;
    }
    for (int n = 0; n <= N; ++n) {
        double lw = lgamma((double)N + 1.0) - lgamma((double)n + 1.0)
                  - lgamma((double)(N - n) + 1.0) - (double)N * log(2.0);
        w[n] = exp(lw);
    }
}

/* Number of terms kept (w_n >= eps: a weight is dropped only when strictly
 * below eps), and the dropped mass sum_{w_n < eps} w_n. */
int oracle_trunc_terms(int N, double eps, double *dropped)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)(N + 1));
    binom_row(N, w);
    int kept = 0;
    double drop = 0.0;
    for (int n = 0; n <= N; ++n) {
        if (w[n] >= eps) kept++;
        else drop += w[n];
    }
    free(w);
    if (dropped) *dropped = drop;
    return kept;
}

/* Truncated kernel phi_eps(t) = sum over kept n of w_n cos(omega_n t). */
double oracle_trunc_kernel(double t, double sigma_r, int N, double eps)
{
    if (N == 0) return 1.0;
    double *w = (double *)malloc(sizeof(double) * (size_t)(N + 1));
    binom_row(N, w);
    double s = sigma_r * sqrt((double)N);
    double acc = 0.0;
    for (int n = 0; n <= N; ++n)
        if (w[n] >= eps) acc += w[n] * cos((double)(2 * n - N) * t / s);
    free(w);
    return acc;
}

/* Smallest order N for which the polynomial kernel below is non-negative
 * and unimodal on [-T, T]: its zeros +-sigma_r sqrt(2N) must lie outside,
 * N >= T^2 / (2 sigma_r^2). */
int oracle_poly_order_for(double sigma_r, double T)
{
    double x = T / sigma_r;
    return (int)ceil(0.5 * x * x);
}

/* Polynomial range kernel phi(t) = (1 - t^2 / (2 N sigma_r^2))^N; Section 3,
 * p_N, in the scaling of eq. (5).  N = 0 gives phi = 1.  Outside the support
 * |t| <= sigma_r sqrt(2N) the polynomial is evaluated as it stands. */
double oracle_poly_kernel(double t, double sigma_r, int N)
{
    if (N == 0) return 1.0;
    double u = t / sigma_r;
    return ipow(1.0 - u * u / (2.0 * (double)N), N);
}

/* Kernel selector: exact raised cosine, its truncated expansion, or the
 * polynomial kernel.  The truncated kernel is tabulated once per call
 * (weights and frequencies). */
typedef struct {
    int mode;          /* 0: cos^N, 1: truncated sum, 2: polynomial */
    int N;
    double sigma_r;
    int nterm;
    double *w;
    double *om;
} kern_t;

static void kern_init(kern_t *k, double sigma_r, int N, double eps, int truncated)
{
    memset(k, 0, sizeof(*k));
    k->N = N;
    k->sigma_r = sigma_r;
    k->mode = (truncated && N > 0) ? 1 : 0;
    if (k->mode == 1) {
        k->w = (double *)malloc(sizeof(double) * (size_t)(N + 1));
        k->om = (double *)malloc(sizeof(double) * (size_t)(N + 1));
        double s = sigma_r * sqrt((double)N);
        double *wr = (double *)malloc(sizeof(double) * (size_t)(N + 1));
        binom_row(N, wr);
        for (int n = 0; n <= N; ++n) {
            double w = wr[n];
            if (w >= eps) {
                k->w[k->nterm] = w;
                k->om[k->nterm] = (double)(2 * n - N) / s;
                k->nterm++;
            }
        }
        free(wr);
    }
}

static void kern_free(kern_t *k)
{
    free(k->w);
    free(k->om);
}

static inline double kern_eval(const kern_t *k, double t)
{
    if (k->mode == 0) return oracle_kernel(t, k->sigma_r, k->N);
    if (k->mode == 2) return oracle_poly_kernel(t, k->sigma_r, k->N);
    double acc = 0.0;
    for (int n = 0; n < k->nterm; ++n) acc += k->w[n] * cos(k->om[n] * t);
    return acc;
}

static inline long lmax(long a, long b) { return a > b ? a : b; }
static inline long lmin(long a, long b) { return a < b ? a : b; }

/* P, Q at one pixel by direct summation over the truncated window. */
static void window_pq(const double *f, long H, long W, long r, const kern_t *k,
                      long i, long j, double *P, double *Q)
{
    double fx = f[i * W + j];
    double p = 0.0, q = 0.0;
    long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
    long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
    for (long y = y0; y <= y1; ++y) {
        const double *row = f + y * W;
        for (long x = x0; x <= x1; ++x) {
            double fy = row[x];
            double kv = kern_eval(k, fy - fx);
            p += kv * fy;
            q += kv;
        }
    }
    *P = p;
    *Q = q;
}

static double *widen(const float *f, long n)
{
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    for (long i = 0; i < n; ++i) d[i] = (double)f[i];
    return d;
}

static long clamp_radius(long r, long H, long W)
{
    long m = H > W ? H : W;
    return r > m ? m : r;
}

/* Full image, double input.  out, P, Q may be NULL (each independently). */
void oracle_bilateral_f64(const double *f, int H, int W, int radius, double sigma_r, int N,
                          double eps, int truncated, double *out, double *P, double *Q)
{
    kern_t k;
    kern_init(&k, sigma_r, N, eps, truncated);
    long r = clamp_radius(radius, H, W);
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < H; ++i) {
        for (long j = 0; j < W; ++j) {
            double p, q;
            window_pq(f, H, W, r, &k, i, j, &p, &q);
            if (out) out[i * W + j] = p / q;
            if (P) P[i * W + j] = p;
            if (Q) Q[i * W + j] = q;
        }
    }
    kern_free(&k);
}

/* Full image, float input (widened exactly). */
void oracle_bilateral(const float *f, int H, int W, int radius, double sigma_r, int N,
                      double eps, int truncated, double *out, double *P, double *Q)
{
    double *d = widen(f, (long)H * W);
    oracle_bilateral_f64(d, H, W, radius, sigma_r, N, eps, truncated, out, P, Q);
    free(d);
}

/* Selected pixels only (flat row-major indices), float input read in place. */
void oracle_bilateral_at(const float *f, int H, int W, int radius, double sigma_r, int N,
                         double eps, int truncated, const long long *idx, long long n,
                         double *out, double *P, double *Q)
{
    kern_t k;
    kern_init(&k, sigma_r, N, eps, truncated);
    long r = clamp_radius(radius, H, W);
#pragma omp parallel
    {
#pragma omp for schedule(dynamic, 64)
        for (long long s = 0; s < n; ++s) {
            long i = (long)(idx[s] / W), j = (long)(idx[s] % W);
            double fx = (double)f[i * (long)W + j];
            double p = 0.0, q = 0.0;
            long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
            long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
            for (long y = y0; y <= y1; ++y) {
                const float *row = f + y * (long)W;
                for (long x = x0; x <= x1; ++x) {
                    double fy = (double)row[x];
                    double kv = kern_eval(&k, fy - fx);
                    p += kv * fy;
                    q += kv;
                }
            }
            if (out) out[s] = p / q;
            if (P) P[s] = p;
            if (Q) Q[s] = q;
        }
    }
    kern_free(&k);
}

/*
 * Gradient of a scalar loss L(out) given gbar = dL/d out, by hand through the
 * definition above (exact raised cosine, N held fixed):
 *   dL/df(z) = sum_{x in B(z)} a(x) [phi(f_z - f_x) + phi'(f_z - f_x)(f_z - u_x)]
 *              - a(z) sum_{y in B(z)} phi'(f_y - f_z)(f_y - u_z)
 *   dL/dsigma_r = -(1/sigma_r) sum_x a(x) sum_{y in B(x)} (f_y - f_x) phi'(f_y - f_x)(f_y - u_x)
 * with a = gbar / Q, u = P / Q.  The first sum uses the symmetry of window
 * membership (z in B(x) iff x in B(z)).  The sigma_r derivative uses
 * d phi / d sigma_r = -(t / sigma_r) phi'(t).  grad_f and grad_sigma may be
 * NULL independently.  The sigma_r sum is reduced per row, then over rows in
 * order, so it does not depend on the thread count.
 */
void oracle_bilateral_grad_f64(const double *f, const double *gbar, int H, int W, int radius,
                               double sigma_r, int N, double *grad_f, double *grad_sigma,
                               double *u_out)
{
    long n = (long)H * W;
    long r = clamp_radius(radius, H, W);
    kern_t k;
    kern_init(&k, sigma_r, N, 0.0, 0);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    double *s1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *rowsum = (double *)calloc((size_t)H, sizeof(double));

#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < H; ++i) {
        for (long j = 0; j < W; ++j) {
            double p, q;
            window_pq(f, H, W, r, &k, i, j, &p, &q);
            u[i * W + j] = p / q;
            a[i * W + j] = gbar[i * W + j] / q;
        }
    }

#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < H; ++i) {
        double racc = 0.0;
        for (long j = 0; j < W; ++j) {
            double fx = f[i * W + j], ux = u[i * W + j];
            double t1 = 0.0, t2 = 0.0;
            long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
            long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
            for (long y = y0; y <= y1; ++y) {
                for (long x = x0; x <= x1; ++x) {
                    double fy = f[y * W + x];
                    double d = fy - fx;
                    double dp = oracle_kernel_deriv(d, sigma_r, N);
                    t1 += dp * (fy - ux);
                    t2 += d * dp * (fy - ux);
                }
            }
            s1[i * W + j] = t1;
            racc += a[i * W + j] * t2;
        }
        rowsum[i] = racc;
    }

    if (grad_f) {
#pragma omp parallel for schedule(dynamic, 1)
        for (long i = 0; i < H; ++i) {
            for (long j = 0; j < W; ++j) {
                double fz = f[i * W + j];
                double acc = 0.0;
                long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
                long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
                for (long y = y0; y <= y1; ++y) {
                    for (long x = x0; x <= x1; ++x) {
                        long xi = y * W + x;
                        double d = fz - f[xi];
                        acc += a[xi] * (oracle_kernel(d, sigma_r, N)
                                        + oracle_kernel_deriv(d, sigma_r, N) * (fz - u[xi]));
                    }
                }
                grad_f[i * W + j] = acc - a[i * W + j] * s1[i * W + j];
            }
        }
    }
    if (grad_sigma) {
        double tot = 0.0;
        for (long i = 0; i < H; ++i) tot += rowsum[i];
        *grad_sigma = -tot / sigma_r;
    }
    if (u_out) memcpy(u_out, u, sizeof(double) * (size_t)n);
    free(u);
    free(a);
    free(s1);
    free(rowsum);
    kern_free(&k);
}

/*
 * Spatial kernel of Algorithms 1 and 2 with M > 1 (Section 2, eq. (2) and
 * eq. (3) with a non-trivial spatial kernel; Section 3, separable kernels):
 * the product w(y_1 - x_1) w(y_2 - x_2) of one-dimensional raised cosines
 *     w(d) = [cos(d / (sigma_s sqrt(Ns)))]^Ns,
 * i.e. q_Ns of Section 3 in the scaling of eq. (6), whose Gaussian limit has
 * standard deviation sigma_s (eq. (7) for the separable product).  Ns = 0
 * gives w = 1, the box of the functions above.  The window B(x) is the same
 * truncated (2r+1)^2 square.
 */
double oracle_spatial_weight(double d, double sigma_s, int Ns)
{
    if (Ns == 0) return 1.0;
    double a = d / (sigma_s * sqrt((double)Ns));
    return ipow(cos(a), Ns);
}

/* P, Q at one pixel with the spatial weights ws[d + r], d = -r .. r. */
static void window_pq_sp(const double *f, long H, long W, long r, const kern_t *k, const double *ws,
                         long i, long j, double *P, double *Q)
{
    double fx = f[i * W + j];
    double p = 0.0, q = 0.0;
    long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
    long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
    for (long y = y0; y <= y1; ++y) {
        const double *row = f + y * W;
        double wy = ws[y - i + r];
        for (long x = x0; x <= x1; ++x) {
            double fy = row[x];
            double kv = wy * ws[x - j + r] * kern_eval(k, fy - fx);
            p += kv * fy;
            q += kv;
        }
    }
    *P = p;
    *Q = q;
}

static double *spatial_table(long r, double sigma_s, int Ns)
{
    double *ws = (double *)malloc(sizeof(double) * (size_t)(2 * r + 1));
    for (long d = -r; d <= r; ++d) ws[d + r] = oracle_spatial_weight((double)d, sigma_s, Ns);
    return ws;
}

/* Full image with the separable spatial kernel, double input; out, P, Q may
 * be NULL independently.  N = 0 makes the range kernel 1: Algorithm 1, the
 * normalised linear spatial filter. */
void oracle_bilateral_sp_f64(const double *f, int H, int W, int radius, double sigma_r, int N,
                             double sigma_s, int Ns, double *out, double *P, double *Q)
{
    kern_t k;
    kern_init(&k, sigma_r, N, 0.0, 0);
    long r = clamp_radius(radius, H, W);
    double *ws = spatial_table(r, sigma_s, Ns);
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < H; ++i) {
        for (long j = 0; j < W; ++j) {
            double p, q;
            window_pq_sp(f, H, W, r, &k, ws, i, j, &p, &q);
            if (out) out[i * W + j] = p / q;
            if (P) P[i * W + j] = p;
            if (Q) Q[i * W + j] = q;
        }
    }
    free(ws);
    kern_free(&k);
}

/* The same, float input (widened exactly). */
void oracle_bilateral_sp(const float *f, int H, int W, int radius, double sigma_r, int N,
                         double sigma_s, int Ns, double *out, double *P, double *Q)
{
    double *d = widen(f, (long)H * W);
    oracle_bilateral_sp_f64(d, H, W, radius, sigma_r, N, sigma_s, Ns, out, P, Q);
    free(d);
}

/* The same at selected pixels (flat row-major indices). */
void oracle_bilateral_sp_at(const float *f, int H, int W, int radius, double sigma_r, int N,
                            double sigma_s, int Ns, const long long *idx, long long n,
                            double *out, double *P, double *Q)
{
    kern_t k;
    kern_init(&k, sigma_r, N, 0.0, 0);
    long r = clamp_radius(radius, H, W);
    double *ws = spatial_table(r, sigma_s, Ns);
#pragma omp parallel
    {
#pragma omp for schedule(dynamic, 64)
        for (long long s = 0; s < n; ++s) {
            long i = (long)(idx[s] / W), j = (long)(idx[s] % W);
            double fx = (double)f[i * (long)W + j];
            double p = 0.0, q = 0.0;
            long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
            long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
            for (long y = y0; y <= y1; ++y) {
                const float *row = f + y * (long)W;
                double wy = ws[y - i + r];
                for (long x = x0; x <= x1; ++x) {
                    double fy = (double)row[x];
                    double kv = wy * ws[x - j + r] * kern_eval(&k, fy - fx);
                    p += kv * fy;
                    q += kv;
                }
            }
            if (out) out[s] = p / q;
            if (P) P[s] = p;
            if (Q) Q[s] = q;
        }
    }
    free(ws);
    kern_free(&k);
}

/* ---- polynomial range kernel (box spatial kernel) ---- */

static void kern_init_poly(kern_t *k, double sigma_r, int N)
{
    memset(k, 0, sizeof(*k));
    k->N = N;
    k->sigma_r = sigma_r;
    k->mode = 2;
}

/* Full image with the polynomial range kernel, double input; out, P, Q may be
 * NULL independently. */
void oracle_bilateral_poly_f64(const double *f, int H, int W, int radius, double sigma_r, int N,
                               double *out, double *P, double *Q)
{
    kern_t k;
    kern_init_poly(&k, sigma_r, N);
    long r = clamp_radius(radius, H, W);
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < H; ++i) {
        for (long j = 0; j < W; ++j) {
            double p, q;
            window_pq(f, H, W, r, &k, i, j, &p, &q);
            if (out) out[i * W + j] = p / q;
            if (P) P[i * W + j] = p;
            if (Q) Q[i * W + j] = q;
        }
    }
}

/* The same with float input (widened exactly). */
void oracle_bilateral_poly(const float *f, int H, int W, int radius, double sigma_r, int N,
                           double *out, double *P, double *Q)
{
    double *d = widen(f, (long)H * W);
    oracle_bilateral_poly_f64(d, H, W, radius, sigma_r, N, out, P, Q);
    free(d);
}

/* Selected pixels only (flat row-major indices), float input. */
void oracle_bilateral_poly_at(const float *f, int H, int W, int radius, double sigma_r, int N,
                              const long long *idx, long long n, double *out)
{
    kern_t k;
    kern_init_poly(&k, sigma_r, N);
    long r = clamp_radius(radius, H, W);
#pragma omp parallel for schedule(dynamic, 64)
    for (long long s = 0; s < n; ++s) {
        long i = (long)(idx[s] / W), j = (long)(idx[s] % W);
        double fx = (double)f[i * (long)W + j];
        double p = 0.0, q = 0.0;
        long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
        long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
        for (long y = y0; y <= y1; ++y) {
            const float *row = f + y * (long)W;
            for (long x = x0; x <= x1; ++x) {
                double fy = (double)row[x];
                double kv = kern_eval(&k, fy - fx);
                p += kv * fy;
                q += kv;
            }
        }
        out[s] = p / q;
    }
}

/* ---- two-pixel-patch non-local means (Section 5, p = 2) ----
 *
 * For pixel x and window pixel y in B(x) (the truncated (2r+1)^2 square):
 *     t_1 = f(x) - f(y),   t_2 = fe(x + u) - fe(y + u),
 *     phi(t_1, t_2) = [cos(t_1 / (sigma_1 sqrt N_1))]^N_1 [cos(t_2 / (sigma_2 sqrt N_2))]^N_2,
 *     out(x) = sum_y phi f(y) / sum_y phi,
 * where u = (uy, ux) is the second patch pixel's offset and fe extends f
 * beyond the image by its nearest border pixel (the paper does not discuss
 * borders; this reading keeps every patch complete).  Each factor is the
 * raised cosine of eq. (6) with its own scale: the Gaussian
 * exp(-h^-2 (g_1 t_1^2 + g_2 t_2^2)) of the Discussion has sigma_k =
 * h / sqrt(2 g_k).  N_k = 0 makes factor k equal to 1. */
static inline double ext(const double *f, long H, long W, long i, long j)
{
    i = i < 0 ? 0 : (i >= H ? H - 1 : i);
    j = j < 0 ? 0 : (j >= W ? W - 1 : j);
    return f[i * W + j];
}

static void window_pq_nlm2(const double *f, long H, long W, long r, double s1, int N1, double s2, int N2,
                           long uy, long ux, long i, long j, double *P, double *Q)
{
    double fx = f[i * W + j];
    double gx = ext(f, H, W, i + uy, j + ux);
    double p = 0.0, q = 0.0;
    long y0 = lmax(0, i - r), y1 = lmin(H - 1, i + r);
    long x0 = lmax(0, j - r), x1 = lmin(W - 1, j + r);
    for (long y = y0; y <= y1; ++y) {
        for (long x = x0; x <= x1; ++x) {
            double fy = f[y * W + x];
            double gy = ext(f, H, W, y + uy, x + ux);
            double kv = oracle_kernel(fy - fx, s1, N1) * oracle_kernel(gy - gx, s2, N2);
            p += kv * fy;
            q += kv;
        }
    }
    *P = p;
    *Q = q;
}

/* Full image, double input; out, P, Q may be NULL independently. */
void oracle_nlm2_f64(const double *f, int H, int W, int radius, double sigma_1, int N1, double sigma_2, int N2,
                     int uy, int ux, double *out, double *P, double *Q)
{
    long r = clamp_radius(radius, H, W);
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < H; ++i) {
        for (long j = 0; j < W; ++j) {
            double p, q;
            window_pq_nlm2(f, H, W, r, sigma_1, N1, sigma_2, N2, uy, ux, i, j, &p, &q);
            if (out) out[i * W + j] = p / q;
            if (P) P[i * W + j] = p;
            if (Q) Q[i * W + j] = q;
        }
    }
}

/* The same with float input (widened exactly). */
void oracle_nlm2(const float *f, int H, int W, int radius, double sigma_1, int N1, double sigma_2, int N2,
                 int uy, int ux, double *out, double *P, double *Q)
{
    double *d = widen(f, (long)H * W);
    oracle_nlm2_f64(d, H, W, radius, sigma_1, N1, sigma_2, N2, uy, ux, out, P, Q);
    free(d);
}

/* Selected pixels only (flat row-major indices), float input. */
void oracle_nlm2_at(const float *f, int H, int W, int radius, double sigma_1, int N1, double sigma_2, int N2,
                    int uy, int ux, const long long *idx, long long n, double *out)
{
    double *d = widen(f, (long)H * W);
    long r = clamp_radius(radius, H, W);
#pragma omp parallel for schedule(dynamic, 64)
    for (long long s = 0; s < n; ++s) {
        long i = (long)(idx[s] / W), j = (long)(idx[s] % W);
        double p, q;
        window_pq_nlm2(d, H, W, r, sigma_1, N1, sigma_2, N2, uy, ux, i, j, &p, &q);
        out[s] = p / q;
    }
    free(d);
}

int oracle_num_threads(void)
{
    return omp_get_max_threads();
}
