/*
 * bsk.h — C ABI of libbsk: constant-time bilateral filtering with shiftable
 * kernels on AMD Instinct MI355X (gfx950).
 *
 * Method (K. N. Chaudhury, "Constant-time filtering using shiftable kernels"):
 * eq. (3) of Section 2 defines the bilateral filter
 *     out(x) = sum_{y in B(x)} phi(f(y) - f(x)) f(y)  /  sum_{y in B(x)} phi(f(y) - f(x)).
 * B(x) is the (2r+1)x(2r+1) square centred at x, truncated at the image
 * border (pixels outside the image are absent).  The spatial kernel is a box
 * by default (every pixel of B(x) has weight 1); bsk_options selects instead
 * the separable raised cosine of Section 3 (Algorithm 2 with M > 1 spatial
 * basis functions, and Algorithm 1 when the range order is 0).
 * The range kernel is the raised cosine q_N of Section 3 in the scaling of
 * Theorem 3.3, eq. (6): phi(t) = cos^N(t / (sigma_r sqrt N)), which tends to
 * the Gaussian exp(-t^2 / 2 sigma_r^2).  Being a finite sum of N+1 complex
 * exponentials (Section 1), phi is shiftable, so Algorithm 2 computes the
 * filter exactly (up to rounding) from O(1)-per-pixel moving sums
 * (Section 2, Sum(F, x, T)) of pointwise transforms of f.  bsk_options can
 * select instead Section 3's polynomial kernel p_N in the scaling of eq. (5),
 * (1 - t^2 / (2 N sigma_r^2))^N, also exact up to rounding (polynomials are
 * shiftable).
 *
 * T is the range bound of Section 3 (values are assumed to span at most T).
 * It only selects the automatic order N_0 = ceil((2T / (pi sigma_r))^2), the
 * smallest order for which phi is non-negative and unimodal on [-T, T]
 * (Section 3.1: N_0 = O(T^2 / sigma^2)).
 *
 * Conventions for every entry point:
 *   - Image pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors),
 *     row-major, H rows of W elements, element pitch = W unless a pitch is
 *     given in bsk_options.  The caller owns every buffer.
 *   - The library never allocates the caller's outputs.  It may allocate a
 *     device workspace (cached per device, released by bsk_release()).
 *   - Every call that takes a `stream` (a hipStream_t; NULL = the default
 *     stream) is asynchronous on that stream.  bilateral_shiftable() uses the
 *     default stream and returns after its work completes.
 *   - Errors are returned as bsk_status codes, never thrown; bsk_last_error()
 *     returns a thread-local message for the last failing call.  Arguments are
 *     validated before any work is queued: on an error nothing is launched.
 *     Faults inside a kernel surface at the next synchronising call.
 *   - Preconditions that are not checked: inputs are finite (a NaN spreads
 *     along the running sums of its row strip); input and output buffers do
 *     not overlap except where an argument says so.
 *   - radius may exceed the image: the window is clamped to the image, so
 *     radius >= max(H, W) - 1 gives the whole-image filter.  Radii whose
 *     clamped value exceeds BSK_MAX_RADIUS are rejected with BSK_EUNSUPPORTED.
 */
#ifndef BSK_H
#define BSK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSK_OK = 0,
    BSK_EINVAL = -1,        /* bad argument (null pointer, size, non-finite sigma_r/T, ...) */
    BSK_ERANGE = -2,        /* order too large (more than BSK_MAX_ORDERS folded orders) */
    BSK_ENOMEM = -3,        /* workspace allocation failed */
    BSK_EHIP = -4,          /* HIP runtime error (no device, launch failure, ...) */
    BSK_EUNSUPPORTED = -5   /* valid request the library does not handle */
} bsk_status;

typedef enum {
    BSK_FP32 = 0,   /* FP32 data, FP32 transforms, sums and recombination */
    BSK_BF16 = 1,   /* precision form: stack quantised to bfloat16, FP32 sums */
    BSK_FP16 = 2,   /* precision form: stack quantised to float16, FP32 sums */
    BSK_FP64 = 3,   /* FP64 data and arithmetic end to end (img/out are double*) */
    BSK_I16 = 4     /* precision form: stack quantised to 16-bit fixed point (Q15), FP32 sums */
} bsk_precision;

/* Range kernel (Section 3): the raised cosine q_N (default) or the polynomial p_N. */
typedef enum {
    BSK_RANGE_COS = 0,   /* phi(t) = cos^N(t / (sigma_r sqrt N)), eq. (6) scaling */
    BSK_RANGE_POLY = 1   /* phi(t) = (1 - t^2 / (2 N sigma_r^2))^N, eq. (5) scaling */
} bsk_range_kernel;

#define BSK_MAX_ORDERS 256     /* folded orders after truncation: N <= 511 untruncated */
#define BSK_MAX_POLY_ORDER 4096 /* largest N of the polynomial range kernel */
#define BSK_MAX_RADIUS 500     /* clamped radius limit of the fused kernels */

/* Options; a zero-initialised struct means: automatic N_0, FP32, no
 * truncation, no compensation, dense pitch, tuned launch shape, box spatial
 * kernel. */
typedef struct {
    int order_mode;       /* 0: N = N_0 from sigma_r and T; 1: use `N` below */
    int N;                /* range-kernel order when order_mode == 1 (N = 0 is the box mean) */
    int precision;        /* bsk_precision */
    double weight_eps;    /* drop binomial weights 2^-N C(N,n) < weight_eps (Section 3.1); 0 keeps all */
    int kahan;            /* 1: Kahan-compensated FP32 vertical running sums */
    int pitch_in;         /* input row pitch in elements; 0 = W */
    int pitch_out;        /* output row pitch in elements; 0 = W */
    int block;            /* lanes per workgroup (256, 512, 1024); 0 = auto */
    int strip_h;          /* output rows per workgroup; 0 = auto */
    int order_chunk;      /* orders per pass, one of the pass sizes of the kernel that runs:
                             FP32 forward 256: 24|20|16|12|8 (12: plain FP32 stack only; 24
                             and 20: plain FP32 stack at radii 1 to 64), 512: 8|4,
                             1024: 4|2 (lanes: full|half); adjoint 256: 24|16|12|8, 512: 8|4,
                             1024: 2|1; batched 256: 16|12|8, 512: 8|4, 1024: 4|2; spatial kernel 4|2
                             (one frequency) or 2|1; polynomial range kernel (channel pairs)
                             256: 24|16|8 (24 at the radii 3, 5, 8, 10, 16, 20, 25, 32), 512:
                             16|8, 1024: 8|4; ignored by FP64 and the training
                             forward; 0 = automatic (the cheaper for the order count) */
    /* Spatial kernel (Algorithms 1 and 2 with M > 1; Section 3, separable
     * kernels): 0 = the box; Ns in 1..6 = the separable raised cosine
     * w(dy) w(dx), w(d) = cos^Ns(d / (spatial_sigma sqrt Ns)) on the same
     * (2r+1)^2 window (spatial basis of M = (Ns+1)^2 functions); -1 = the
     * smallest Ns keeping w non-negative and unimodal on [-r, r],
     * ceil((2r / (pi spatial_sigma))^2), which must not exceed 6.  The
     * paper's q_Ns(t) = cos^Ns(pi t / 2T_s) is spatial_sigma = 2 T_s / (pi sqrt Ns).
     * Supported by the plain FP32 forward (bilateral_shiftable_ex) with
     * 256- or 512-lane strips; the other entry points return BSK_EUNSUPPORTED. */
    int spatial_N;
    double spatial_sigma; /* > 0 when spatial_N != 0 */
    /* Range kernel (bsk_range_kernel).  BSK_RANGE_POLY selects Section 3's
     * p_N in the scaling of eq. (5): phi(t) = (1 - t^2 / (2 N sigma_r^2))^N,
     * which tends to exp(-t^2 / 2 sigma_r^2) like the raised cosine.  Its
     * automatic order (order_mode 0) is N_p = ceil(T^2 / (2 sigma_r^2)), the
     * smallest keeping it non-negative and unimodal on [-T, T]; N is at most
     * BSK_MAX_POLY_ORDER.  The filter is computed from box sums of the
     * Chebyshev polynomials T_k of the values normalised to [-1, 1] (a
     * polynomial basis, hence exact up to rounding); weight_eps > 0 drops the
     * coefficients of the kernel's Chebyshev expansion past the point where
     * their largest magnitudes sum to at most weight_eps (bsk_poly_plan_info).
     * Supported: bilateral_shiftable_ex with BSK_FP32 or BSK_FP64, the box
     * spatial kernel, no compensation; other requests return
     * BSK_EUNSUPPORTED.  Precondition: the values each workgroup reads (its
     * strip of columns and rows within r of its output rows) span at most T;
     * beyond it the channels grow without bound. */
    int range_kernel;
} bsk_options;

/*
 * Bilateral filter of one FP32 image (eq. (3), Algorithm 2 with a box spatial
 * kernel and the raised-cosine range kernel at order N_0(sigma_r, T)).
 *   img:    device, H*W floats, row-major (read only)
 *   out:    device, H*W floats (written); must not overlap img
 *   radius: box half-width r >= 0 (window (2r+1)^2)
 *   sigma_r > 0: range scale (the Gaussian limit's standard deviation)
 *   T > 0:  range bound, selects N_0
 * Runs on the default stream and synchronises before returning.
 * Performance: with 256-lane strips (the default for r <= 64) every radius
 * from 1 to 64 runs kernels compiled for that radius in the plain FP32
 * forward and the training forward below, every radius from 1 to 32 in the
 * adjoint, and the radii 3, 5, 8, 10, 16, 20, 25 and 32 also in the q_2
 * spatial kernel, the FP32 polynomial kernel and the two-pixel patch's
 * 16-order pass.  They are 3-10% faster than the run-time-radius kernels the
 * other radii use; the results agree to FP32 rounding.
 */
int bilateral_shiftable(const float *img, int H, int W, int radius, float sigma_r, float T,
                        float *out);

/*
 * As bilateral_shiftable, with options and a stream (asynchronous).
 * img/out are float* for BSK_FP32/BF16/FP16/I16 and double* for BSK_FP64.
 * opt may be NULL (defaults).  If opt->weight_eps > 0, folded orders whose
 * unfolded weight is below it are dropped (Section 3.1); the dropped mass is
 * reported by bsk_plan_info().  A weight_eps that drops every order is
 * BSK_EINVAL (the filter would be 0/0).
 */
int bilateral_shiftable_ex(const void *img, int H, int W, int radius, float sigma_r, float T,
                           void *out, const bsk_options *opt, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter as bilateral_shiftable_ex, with the same kernels and launch shapes,
 * making no device allocation.  The partial accumulators of a multi-pass
 * launch (more folded orders than one pass holds) live in a fixed 128 MiB
 * device array of the library instead of the per-stream workspace: two FP32
 * planes of up to 4096 x 4096 pixels, or two FP64 planes of up to 4096 x 2048.
 *   img, out, H, W, radius, sigma_r, T, opt, stream: as bilateral_shiftable_ex
 * Supported: the raised-cosine range kernel with the box spatial kernel, in
 * every precision; the separable spatial kernel and the polynomial range
 * kernel return BSK_EUNSUPPORTED.  A multi-pass request whose accumulators
 * exceed the array returns BSK_ENOMEM before anything is queued.
 * Each device holds one copy of the array, from the first call on it until
 * the process ends, and every call on a device shares it: calls that overlap
 * in time on one device (on different streams, or from different threads)
 * race and must be ordered by the caller.  Nothing in the array needs to start
 * at zero.
 */
int bilateral_shiftable_noalloc(const void *img, int H, int W, int radius, float sigma_r, float T,
                                void *out, const bsk_options *opt, void *stream);

/*
 * Two-pixel-patch non-local means (Section 5, the Discussion, with p = 2
 * patch pixels u_1 = 0 and u_2 = (uy, ux)): the bilateral filter of eq. (3)
 * with the range kernel comparing the patches {x, x + u_2} and {y, y + u_2},
 *     phi = cos^N1(t_1 / (sigma_1 sqrt N1)) cos^N2(t_2 / (sigma_2 sqrt N2)),
 *     t_1 = f(x) - f(y),   t_2 = f(x + u_2) - f(y + u_2),
 * the separable shiftable approximation of the Discussion's anisotropic
 * Gaussian exp(-h^-2 (g_1 t_1^2 + g_2 t_2^2)) (sigma_k = h / sqrt(2 g_k)).
 * Patch pixels beyond the image read its nearest border pixel; the window
 * B(x) is the truncated (2r+1)^2 square of the box kernel.  The expansion has
 * (N1 + 1) times the folded orders of N2 terms (the order grows as n^p, which
 * is why larger patches are not offered).
 *   img, out:  device FP32, as for bilateral_shiftable_ex (must not overlap)
 *   N1, N2:    orders, or < 0 for N_0(sigma_k, T); at most 1000 each
 *   opt:       NULL or options with order_mode 0, FP32, no compensation, the
 *              box spatial kernel and the raised cosine; weight_eps > 0 drops
 *              terms of either factor whose binomial weight is below it
 *              (BSK_EINVAL if that drops every term of a factor);
 *              pitches, block, strip_h and order_chunk as for the forward
 * When the second pixel's folded orders fit in one pass of order_chunk
 * orders, several first-pixel terms share each pass; otherwise each spans
 * whole passes of its own.
 * Asynchronous on `stream`.  BSK_ERANGE when more than 65536 terms remain.
 */
int bilateral_shiftable_nlm2(const float *img, int H, int W, int radius, float sigma_1, float sigma_2, int N1,
                             int N2, int uy, int ux, float T, float *out, const bsk_options *opt, void *stream);

/*
 * Training forward (FP32): the filter output plus what the adjoint needs.
 *   out:   device H*W floats: u = P/Q
 *   saved: device 3*H*W floats, planar: Q (the normaliser eta of eq. (3)),
 *          E1(z) = sum_{y in B(z)} phi'(f_y - f_z)(f_y - u_z),
 *          E2(x) = sum_{y in B(x)} (f_y - f_x) phi'(f_y - f_x)(f_y - u_x).
 * opt may be NULL; only FP32 is supported (BSK_EUNSUPPORTED otherwise).
 */
int bilateral_shiftable_train(const float *img, int H, int W, int radius, float sigma_r, float T,
                              const bsk_options *opt, float *out, float *saved, void *stream);

/*
 * Adjoint of the filter (FP32), by differentiating eq. (3) through the
 * shiftable expansion: the adjoint of a box moving sum is a box moving sum,
 * so d/df is again one pass of Algorithm 2 over the channels
 * (a cos, a sin, a u cos, a u sin), a = grad_out / Q.  N is held fixed.
 *   img:       device H*W input image
 *   grad_out:  device H*W, dL/d out
 *   out,saved: from bilateral_shiftable_train on the same img and parameters;
 *              both NULL makes the call recompute them into the workspace
 *   grad_img:  device H*W (written), or NULL to skip
 *   grad_sigma: device pointer to ONE float (written: dL/d sigma_r), or NULL.
 *              The reduction is deterministic (fixed order, no atomics).
 */
int bilateral_shiftable_backward(const float *img, const float *grad_out, const float *out,
                                 const float *saved, int H, int W, int radius, float sigma_r,
                                 float T, const bsk_options *opt, float *grad_img,
                                 float *grad_sigma, void *stream);

/*
 * The training forward and the adjoint above for a stack of B images of one
 * size, filtered with one set of parameters, each in ONE launch (the tiles of
 * all images share the grid).  Layout, all dense and device-resident:
 *   img, out, grad_out, grad_img: [B][H][W] floats
 *   saved:                        [B][3][H][W] floats (Q, E1, E2 per image)
 * Each image is filtered exactly as by the single-image call; grad_sigma
 * receives the sum over the stack of dL/d sigma_r (sigma_r is shared, so this
 * is the gradient of the summed loss), reduced in a fixed order.  B >= 1;
 * other arguments and errors as for the single-image calls.
 */
int bilateral_shiftable_train_stack(const float *img, int B, int H, int W, int radius, float sigma_r, float T,
                                    const bsk_options *opt, float *out, float *saved, void *stream);
int bilateral_shiftable_backward_stack(const float *img, const float *grad_out, const float *out,
                                       const float *saved, int B, int H, int W, int radius, float sigma_r, float T,
                                       const bsk_options *opt, float *grad_img, float *grad_sigma, void *stream);

/* One image of a batched call (FP32, device pointers, dense pitch). */
typedef struct {
    const float *img;
    float *out;
    int H, W;
    int radius;
    float sigma_r;
    int N;            /* < 0: N_0(sigma_r, T); >= 0: explicit order */
} bsk_image_desc;

/*
 * Filter B independent images of different sizes, radii and sigma_r in ONE
 * persistent kernel launch.  Each image is filtered exactly as by
 * bilateral_shiftable_ex (eq. (3) through Algorithm 2, box spatial kernel,
 * raised-cosine range kernel of eq. (6) at its own order); gathering many
 * images into one launch has no counterpart in the paper.  descs is a HOST array of B descriptors.  Work
 * units (image, strip, row segment) are claimed from a device work counter.
 * Launch shape: opt->block, opt->strip_h (rows per unit) and opt->order_chunk
 * (orders per pass: the batched kernel's 256/512/1024-lane pass of 16/8/4
 * orders or its half) when non-zero; otherwise the shapes that
 * bsk_autotune_batched measured for the batch's largest radius bucket (lanes)
 * and for each image's (radius bucket, order bucket) (rows, orders per pass);
 * otherwise the defaults (lanes from the largest radius, 96 rows, the pass
 * size that pads fewer orders).  bsk_batched_shape reports the choice.
 * The descriptor table is staged through a library-owned device buffer, so
 * consecutive batched calls on one device must be ordered on one stream.
 */
int bilateral_shiftable_batched(const bsk_image_desc *descs, int B, float T,
                                const bsk_options *opt, void *stream);

/*
 * Batched call recorded once into a HIP graph and replayed: the first call
 * with a given `key` captures the launch (descriptor upload + kernel) on
 * `stream`; later calls with the same key and the same descriptors replay it.
 * Returns BSK_EINVAL if the descriptors differ from the captured ones.
 */
int bilateral_shiftable_batched_graph(const bsk_image_desc *descs, int B, float T,
                                      const bsk_options *opt, int key, void *stream);

/*
 * Launch shape the batched entry points would use for these descriptors and
 * options (host only, nothing is queued): lanes per workgroup, and per
 * descriptor (in the order given) the rows per work unit (at most the image
 * height) and the orders per pass.  block, rows and chunk are nullable; rows
 * and chunk hold B entries.  Errors as for bilateral_shiftable_batched.
 */
int bsk_batched_shape(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, int *block,
                      int *rows, int *chunk);

/*
 * Autotuner of the batched launch (strip and tile sizes of the persistent
 * kernel).  Times bilateral_shiftable_batched on these descriptors (their out
 * buffers are overwritten many times; the stream is synchronised): first the
 * lanes per workgroup that fit the largest radius, then, bucket by bucket
 * (clamped radius bucket 0, 1, 2-3, 4-7, ...; folded-order bucket 1, 2, 3-4,
 * 5-8, ...; buckets with the most pixels first), the rows per work unit in
 * {32, 48, 64, 96, 128, 192, 256} and the two pass sizes, keeping each change
 * that makes the whole launch faster.  The result is stored per bucket and
 * used by later batched calls whose options leave block, strip_h and
 * order_chunk at 0.  opt's block, strip_h and order_chunk are ignored.
 * `path` (nullable) names the JSON-lines cache file (shared with
 * bsk_autotune) that is read first and rewritten with the result.
 * best_block and best_ms (nullable) receive the lanes chosen and the fastest
 * launch time in milliseconds.
 */
int bsk_autotune_batched(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, const char *path,
                         void *stream, int *best_block, double *best_ms);

/* The autotuners' cache (single-image and batched shapes), host only:
 * load adds the entries of a JSON-lines file (BSK_EINVAL if it cannot be
 * read), save writes every entry held (BSK_EINVAL if it cannot be written),
 * clear forgets them all (and stops BSK_TUNE_CACHE from being read later). */
int bsk_tune_cache_load(const char *path);
int bsk_tune_cache_save(const char *path);
int bsk_tune_cache_clear(void);

/* N_0 = ceil((2T / (pi sigma_r))^2) (Section 3.1); -1 on invalid input. */
int bsk_order_for(float sigma_r, float T);

/* Plan of the raised-cosine kernel of order N (Section 3): the binomial
 * theorem expands cos^N into the N+1 terms w_n cos((2n - N) t / (sigma_r sqrt N)),
 * w_n = 2^-N C(N, n); terms n and N - n have equal weights and opposite
 * frequencies and fold into one order (K_full = floor(N/2) + 1 orders).
 * Section 3.1 (its closing paragraph) discards the less significant basis
 * functions: with eps > 0 every unfolded term whose weight is strictly below
 * eps is dropped.
 *   N:       order, 0 .. 1000000
 *   eps:     threshold, finite and >= 0 (0 keeps every term)
 *   K:       (nullable) receives the folded orders kept
 *   dropped: (nullable) receives the dropped unfolded mass sum_{w_n < eps} w_n,
 *            which bounds |phi - phi_eps| everywhere
 * Host only (no device call).  Returns BSK_OK or BSK_EINVAL. */
int bsk_plan_info(int N, double eps, int *K, double *dropped);

/* The dropped mass of bsk_plan_info, sum_{w_n < eps} w_n (Section 3.1's
 * discarded basis functions; 0 if nothing is dropped), or -1.0 for invalid
 * N or eps.  Host only. */
double bsk_truncation_error(int N, double eps);

/* N_p = ceil(T^2 / (2 sigma_r^2)) for the polynomial range kernel; -1 on
 * invalid input. */
int bsk_poly_order_for(float sigma_r, float T);

/* Plan of the polynomial range kernel of order N (N < 0: N_p) for sigma_r, T
 * and truncation eps: the number of Chebyshev coefficients kept (the filter
 * box-sums one more channel than that) and the bound on the dropped part of
 * the normalised kernel, sum over dropped k of max_c |d_k(c)| (0 when eps is
 * 0).  coefs and bound may be NULL.  Returns BSK_OK, BSK_EINVAL or BSK_ERANGE. */
int bsk_poly_plan_info(int N, float sigma_r, float T, double eps, int *coefs, double *bound);

/*
 * Launch-shape autotuner.  Times the candidate shapes (lanes per workgroup in
 * {256, 512, 1024} that fit the radius, the block's pass sizes, output
 * rows per workgroup in {16 .. 256}) of the single-image forward for this exact request on the
 * current device, using the caller's img and out buffers (out is overwritten
 * several times; the stream is synchronised), and caches the fastest.  Later
 * calls with the same clamped radius, folded-order count, H, W and precision,
 * and with opt->block, opt->strip_h and opt->order_chunk all 0, use it.  `path` (nullable)
 * names a JSON-lines cache file that is read first and rewritten with the
 * result; the environment variable BSK_TUNE_CACHE names a file read at first
 * use.  best_block, best_rows, best_chunk and best_ms (nullable) receive the
 * winner.
 */
int bsk_autotune(const void *img, int H, int W, int radius, float sigma_r, float T, void *out,
                 const bsk_options *opt, const char *path, void *stream, int *best_block,
                 int *best_rows, int *best_chunk, double *best_ms);

/*
 * Caps the device memory the library holds as per-stream workspace (the
 * multi-pass accumulator planes, tables and partial sums that the entry
 * points above allocate on first use and keep), per device, in bytes; 0 (the
 * default) removes the cap.  A call whose workspace would exceed the cap
 * fails with BSK_ENOMEM before anything is queued.  Buffers already held are
 * kept (bsk_release() frees them); HIP graphs of the batched entry point own
 * their buffers outside this cap.  Host only; BSK_EINVAL if bytes < 0.
 */
int bsk_set_workspace_limit(long long bytes);

/* Message of the last failing call on this thread ("" if none). */
const char *bsk_last_error(void);

/* Frees every library-owned device buffer and graph. */
int bsk_release(void);

/* Library version string. */
const char *bsk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BSK_H */
