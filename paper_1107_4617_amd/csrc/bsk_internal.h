// Internal declarations shared by the host API and the HIP kernels of libbsk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace bsk {

constexpr int kMaxOrders = 256;   // folded orders a plan may keep
constexpr int kArgOrders = 272;   // weight slots in kernel arguments (kept orders padded to a pass)
constexpr int kMaxSpatialFreq = 3; // non-zero frequencies of the spatial kernel (order Ns <= 6)

// Folded plan of the raised-cosine range kernel (Section 3, q_N, eq. (6)).
// The unfolded expansion cos^N(a) = 2^-N sum_n C(N,n) cos((2n-N) a) pairs
// term n with term N-n (same weight, opposite frequency); after folding, the
// m-th order has frequency omega(m) = omega_base + m * delta (in units of the
// image value) and weight v[m]: twice the unfolded weight, except the zero
// frequency term of even N.  Orders are listed from the lowest frequency
// (largest weight) outwards, so truncation keeps a prefix m < K.
struct Plan {
    int N = 0;
    int K = 0;               // folded orders kept
    int K_full = 0;          // folded orders before truncation
    double gamma = 0.0;      // 1 / sigma_r
    double omega_base = 0.0; // omega(0)
    double delta = 0.0;      // omega(m+1) - omega(m)
    double dropped = 0.0;    // unfolded weight mass removed by truncation
    int start_mode = 0;      // first pass chain start: 0 omega(0) = 0 (even N, N = 0), 1 omega(0) = delta / 2 (odd N)
    double v[kMaxOrders];    // folded weights (FP64)
};

// Builds the plan; returns 0, or -2 if more than kMaxOrders orders remain.
int make_plan(int N, double sigma_r, double eps, Plan *p);

// Folded plan of the separable spatial kernel w(d) = cos^Ns(d / (sigma_s sqrt Ns))
// (Section 3, q_Ns in the scaling of eq. (6)): w(d) = u0 + sum_j u[j] cos(nu[j] d),
// with nu[j] = (Ns - 2j) / (sigma_s sqrt Ns) for j < nsc = ceil(Ns / 2),
// u[j] = 2 * 2^-Ns C(Ns, j), and u0 = 2^-Ns C(Ns, Ns/2) when Ns is even (0 when
// odd).  Ns = 0 is the box (nsc = 0, u0 = 1).
struct SpatialPlan {
    int Ns = 0;
    int nsc = 0;
    bool even = true;
    double sigma = 0.0;
    double u0 = 1.0;
    double u[kMaxSpatialFreq] = {0.0, 0.0, 0.0};
    double nu[kMaxSpatialFreq] = {0.0, 0.0, 0.0};
};
// Returns 0, or -1 if Ns is negative or above 2 kMaxSpatialFreq or sigma_s is not positive.
int make_spatial_plan(int Ns, double sigma_s, SpatialPlan *sp);
int order_for(double sigma_r, double T);
// Full folded-order count and dropped mass without the kMaxOrders limit.
void plan_counts(int N, double eps, int *K, double *dropped);

// Plan of the polynomial range kernel (Section 3, p_N, in the scaling of
// eq. (5)): phi(t) = (1 - t^2 / (2 N sigma_r^2))^N.  Values are mapped to
// x = (f - mu) / rho with rho = T / 2 and mu the midrange of the data a
// workgroup reads, so x lies in [-1, 1] when the data span at most T.  For a
// centre value c the kernel is then g_c(x) = (1 - (x - c)^2 / a^2)^N with
// a = sqrt(2N) sigma_r / rho, a polynomial of degree 2N in x, expanded in
// Chebyshev polynomials: g_c = sum_k d_k(c) T_k(x).  The box sums of the
// channels T_k(x) and x T_k(x) = (T_{k+1} + T_{k-1}) / 2 then give P and Q.
// The coefficients d_k(c) satisfy a five-term recurrence in k (from the
// differential equation h g' = N h' g of g = h^N), run downwards from the
// leading coefficient d_2N in a scaled form d_k = s_k e_k, where s_k is the
// largest |d_k(c)| over c in [-1, 1], so every scaled value stays near 1:
//   e_{k-2} = c alpha_k e_{k-1} + (beta_k + gamma_k c^2) e_k
//             + c delta_k e_{k+1} + epsilon_k e_{k+2},
// started by the row k = 2N + 2, whose only entry is epsilon = (-1)^N, from a
// 1 placed at e_{2N+4}; rows above it shift by four (epsilon = 1).
struct PolyPlan {
    int N = 0;
    int K = 0;               // coefficients kept: d_k for k < K (channels 0 .. K are box-summed)
    double rho = 0.0;        // half-width of the normalised interval (T / 2)
    double ahat = 0.0;       // sqrt(2N) sigma_r / rho
    double bound = 0.0;      // sum over the dropped k of max_c |d_k(c)|: bound on |g_c - kept part|
    double top = 1.0;        // scaled leading coefficient e_2N = (-1)^N
    std::vector<double> lsig;   // ln s_k, k = 0 .. 2N
    // kPolyRow values per k = 0 .. 2N + 2: (alpha, beta, gamma, delta, epsilon) of the
    // step that yields e_{k-2}; rows 0 and 1 are zero (e_{-1} = 0 where a pass needs it)
    std::vector<double> rows;
};
constexpr int kPolyRow = 8;
constexpr int kMaxPolyOrder = 4096;
// Returns 0, or -1 for N < 0 or N > kMaxPolyOrder or a bad sigma_r / T.
int make_poly_plan(int N, double sigma_r, double T, double eps, PolyPlan *pp);
// Smallest N with the polynomial kernel non-negative and unimodal on [-T, T]:
// ceil(T^2 / (2 sigma_r^2)).
int poly_order_for(double sigma_r, double T);

// Buffers and layout of one image as the kernel policies see them.
struct IO {
    const void *img;       // f, float or double, pitch_in elements per row
    const float *aux0;     // backward: dL/dout
    const float *aux1;     // backward: saved Q
    const float *aux2;     // backward: out u
    const float *aux3;     // backward: saved E1
    const float *aux4;     // backward: saved E2
    void *out;             // main output (float or double), pitch_out elements per row
    float *out2;           // train: saved planes Q, E1, E2 (dense)
    int H, W;
    int pitch_in, pitch_out;
    int uy, ux;            // two-pixel patch: offset of the second patch pixel
};

// Per-launch arguments of the single-image strip kernels.  Weights are FP64 in
// the argument block; each kernel converts them to its accumulation type.
struct StripArgs {
    IO io;
    void *ws;              // partial accumulators across order chunks (NACC planes) or null
    double *red;           // backward: per-workgroup partial sums for d/dsigma_r
    int rh, rv;            // clamped horizontal / vertical radii
    int S;                 // output rows per workgroup
    int K;                 // folded orders
    int start_mode;        // 0: omega(0) = 0, 1: omega(0) = delta / 2, 2: general
    int strips;            // workgroups across the width
    double omega_base, delta;
    double v[kArgOrders];  // folded weights, zero past the kept orders
    float vf[kArgOrders];  // the same in FP32
    // separable spatial kernel (unused by the box kernels)
    float sp_u0;
    float sp_u[kMaxSpatialFreq];
    const float *sp_row;   // (cos, sin)(nu_j y), j-major, H rows
    const float *sp_col;   // (cos, sin)(nu_j x), j-major, W columns
    // two-pixel patch (non-local means, Section 5): the orders of one frequency
    // omega_1 = p2_omega1_base + n p2_delta1 of the first patch pixel are the
    // folded orders of the second, laid out in one of two ways (the launch's
    // pack argument):
    //   pack = 0: group n holds p2_group orders (a multiple of the pass size,
    //     zero-weighted beyond the folded ones) and a pass lies within a group;
    //   pack = G > 0: each pass of KR orders holds KR / G groups of G orders,
    //     n = pass (KR / G) + j at positions j G .. j G + G - 1, zero weights
    //     beyond the last group.
    // The weights (FP32, K entries) are in device memory at vf_dev.
    int p2_group;
    double p2_omega1_base, p2_delta1;
    const float *vf_dev;
    // A stack of nimg images of one size and one set of parameters in one launch
    // (0 or 1: a single image).  Image b's buffers start b times the byte stride
    // of each buffer after image 0's: the input, main output, saved planes, the
    // five auxiliary inputs, and the workspace (zero for a null buffer, which
    // stays null).  The tiles of all images share one grid; partial sums in
    // `red` are indexed by the tile over the stack.
    int nimg;
    long long bs_img, bs_out, bs_out2, bs_aux[5], bs_ws;
};

// Tiles of a strip launch: strips x segments per image x images.
inline long long strip_tiles(const StripArgs &a)
{
    return (long long)a.strips * ((a.io.H + a.S - 1) / a.S) * (a.nimg > 1 ? a.nimg : 1);
}

// Per-launch arguments of the polynomial-kernel strip kernel.
struct PolyArgs {
    IO io;
    void *ws;              // across passes: accumulators Q, 2P and four recurrence values
                           // (6 planes of H*W), or null for a single pass
    int rh, rv, S;
    int NP;                // channel pairs, padded to a multiple of the pass size
    int N;
    double rho, inv_rho;   // interval half-width and its inverse
    const void *rows;      // kPolyRow coefficients per k = 0 .. 2 max(N, NP) + 2 (float or
                           // double); past the plan's rows only epsilon = 1 (a shift)
    const void *sig;       // 0, then s_k / s_0 for k < K, then zero: 2 NP + 2 entries
};
hipError_t launch_poly_f32(const PolyArgs &a, int block, int kc, hipStream_t s, int *occ = nullptr);
hipError_t launch_poly_f64(const PolyArgs &a, int block, hipStream_t s, int *occ = nullptr);
int chunk_poly_f32(int block);   // pairs per full pass (the half pass has half)
// The 24-pair pass of the FP32 polynomial kernel (256 lanes at its compile-time
// radii 3, 5, 8, 10, 16, 20, 25 and 32), else 0.
int big_chunk_poly_f32(int block, int rh);
int chunk_poly_f64(int block);

// Launch helpers implemented in bsk_kernels.hip.  `prec` selects the stack
// quantisation (bsk_precision) for the FP32 kernels.  With occ non-null a
// helper launches nothing and stores in *occ the number of workgroups of the
// kernel it would launch that one compute unit holds.
hipError_t launch_forward_f32(const StripArgs &a, int block, int kc, int prec, int kahan, hipStream_t s,
                              int *occ = nullptr);
hipError_t launch_forward_f64(const StripArgs &a, int block, int kc, hipStream_t s, int *occ = nullptr);
// Plain FP32 forward kernels with the radius as a compile-time constant (256
// lanes, radii 1 to 64; bsk_radius.h): whether block and rh have them, and the
// launch (kc one of the 256-lane pass sizes 8, 12, 16, 20 and 24; one pass or
// several).
bool forward_radius_kernel(int block, int rh);
hipError_t launch_forward_f32_radius(const StripArgs &a, int kc, hipStream_t s, int *occ = nullptr);
// The training forward (8-order pass) and the adjoint (24-, 16- and 8-order
// passes) with the radius as a compile-time constant (radii 1 to 32).
bool train_radius_kernel(int block, int rh);
bool backward_radius_kernel(int block, int rh, int kc);
hipError_t launch_train_f32_radius(const StripArgs &a, hipStream_t s, int *occ = nullptr);
hipError_t launch_backward_f32_radius(const StripArgs &a, int kc, hipStream_t s, int *occ = nullptr);
hipError_t launch_train_f32(const StripArgs &a, int block, int kc, hipStream_t s, int *occ = nullptr);
hipError_t launch_backward_f32(const StripArgs &a, int block, int kc, float *grad_sigma, double inv_sigma,
                               int nred, hipStream_t s, int *occ = nullptr);
// FP32 forward of the two-pixel-patch filter (orders per pass kc, one of the
// forward's two pass sizes for the block; pack = 0 or the group size G of the
// packed layout, which needs the 256-lane block and kc = kPatchPackPass).
constexpr int kPatchPackPass = 16;
constexpr int kPatchPackMax = 8;
hipError_t launch_patch2_f32(const StripArgs &a, int block, int kc, int pack, hipStream_t s, int *occ = nullptr);
// The patch kernels with the radius as a compile-time constant
// (bsk_patch_radius.hip): whether block, kc and rh have them, and the launch.
bool patch_radius_kernel(int block, int kc, int rh);
hipError_t launch_patch2_f32_radius(const StripArgs &a, int pack, hipStream_t s, int *occ = nullptr);
// FP32 forward with the separable spatial kernel of plan sp (nsc >= 1).
hipError_t launch_spatial_f32(const StripArgs &a, int block, const SpatialPlan &sp, int kc, hipStream_t s,
                              int *occ = nullptr);
// Fills tab[2 (j n + y) + {0, 1}] = (cos, sin)(nu[j] y) for y < n, j < sp.nsc, in FP64
// with the angle reduced modulo 2 pi before rounding to FP32.
hipError_t launch_phase_table(const SpatialPlan &sp, int n, float *tab, hipStream_t s);
int chunk_spatial_f32(int block, int nsc);         // the full pass
int chunk_spatial_small_f32(int block, int nsc);   // the small pass (the full one where none)
bool spatial_block_ok(int block, int nsc);

// Orders per pass of the strip kernel for a kernel family/block; the FP32
// forward and the adjoint offer a full and a half pass size per block.
bool valid_chunk_forward_f32(int block, int kc);
bool valid_chunk_backward_f32(int block, int kc);
// The 12-order pass of the 256-lane plain FP32 forward and adjoint (0 for
// other lane counts).
int mid_chunk_forward_f32(int block);
// Every pass size of the FP32 forward for a block, stack (prec, kahan) and
// horizontal radius rh: writes them to sizes (at most kMaxForwardChunks) and
// returns how many.  The 256-lane plain stack has 8, 12 and 16 orders, and 20
// and 24 at the compile-time radii; the others the full and the half pass.
constexpr int kMaxForwardChunks = 5;
int forward_chunks_f32(int block, int prec, int kahan, int rh, int *sizes);
bool forward_chunk_ok_f32(int block, int prec, int kahan, int rh, int kc);
int mid_chunk_backward_f32(int block);
int big_chunk_backward_f32(int block);   // 0: none for this lane count
int chunk_forward_f32(int block);
int chunk_forward_f64(int block);
int onepass_chunk_forward_f64(int block);   // 0: none for this lane count
int chunk_train_f32(int block);
int chunk_backward_f32(int block);
int acc_count_forward();   // accumulators per pixel kept across chunks
int acc_count_train();
int acc_count_backward();

// ----------------------------------------------------------------- batched --
struct BatchImage {
    const float *img;
    float *out;
    int H, W, rh, rv, S, K;
    int start_mode;          // as in StripArgs
    int strips;
    int kc;                  // orders per pass: the batched kernel's full pass or its half
    int unit0;               // first work unit of this image
    long long ws_off;        // offset of this image's accumulator planes in ws, -1 if none
    int v_off;               // offset of this image's weights in the weight table
    double omega_base, delta;
};

constexpr int kBatchQueues = 8;   // one work queue per XCD
struct BatchArgs {
    const BatchImage *imgs;  // device table, ordered by unit0
    const double *vtab;      // device folded weights (each image padded to a pass)
    const float *vtabf;      // the same in FP32
    float *ws;               // partial accumulators for images with K > chunk
    int nimg;
    int total_units;
    // Units [qstart[q], qstart[q + 1]) form queue q, served first by the
    // workgroups of XCD q (contiguous runs of units share image rows and columns
    // in that XCD's L2); a workgroup whose queue is empty takes units from the
    // others.  counter holds one claim counter per queue, zeroed by a kernel
    // before each launch.
    int qstart[kBatchQueues + 1];
    unsigned *counter;
};

hipError_t launch_batched_f32(const BatchArgs &a, int block, int grid, hipStream_t s);
int chunk_batched_f32(int block);
int mid_chunk_batched_f32(int block);   // 12 for 256 lanes, else 0
// Largest clamped radius the batched kernel of a given block size accepts.
int max_radius_batched(int block);
int wg_per_cu_batched(int block);

}  // namespace bsk
