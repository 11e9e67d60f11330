// Single-image launches of the fused strip kernels (forward FP32/FP64 and
// precision forms, training forward, adjoint).  The kernel body and its
// design are in bsk_device.h.
#include "bsk_device.h"

namespace bsk {

template <typename AT, int BLOCK, int KC, class POL, int QUANT, bool KAHAN>
__global__ void __launch_bounds__(BLOCK, 1) strip_kernel(const StripArgs a)
{
    constexpr int ROWS = POL::NCH * KC;
    __shared__ AT lds[2 * ROWS * (BLOCK + 1)];
    Geom gm;
    gm.H = a.io.H;
    gm.W = a.io.W;
    gm.pitch_in = a.io.pitch_in;
    gm.pitch_out = a.io.pitch_out;
    gm.rh = a.rh;
    gm.rv = a.rv;
    gm.S = a.S;
    gm.K = a.K;
    gm.omega_base = a.omega_base;
    gm.delta = a.delta;
    gm.v = a.v;
    gm.ws = a.ws;
    strip_body<AT, BLOCK, KC, POL, QUANT, KAHAN>(a.io, gm, blockIdx.x, blockIdx.y, lds, nullptr, nullptr);
}

template <int BLOCK, int KC>
__global__ void __launch_bounds__(BLOCK, 1) backward_kernel(const StripArgs a)
{
    constexpr int ROWS = PolBackward::NCH * KC;
    __shared__ float lds[2 * ROWS * (BLOCK + 1)];
    __shared__ double red_lds[BLOCK];
    Geom gm;
    gm.H = a.io.H;
    gm.W = a.io.W;
    gm.pitch_in = a.io.pitch_in;
    gm.pitch_out = a.io.pitch_out;
    gm.rh = a.rh;
    gm.rv = a.rv;
    gm.S = a.S;
    gm.K = a.K;
    gm.omega_base = a.omega_base;
    gm.delta = a.delta;
    gm.v = a.v;
    gm.ws = a.ws;
    strip_body<float, BLOCK, KC, PolBackward, 0, false>(a.io, gm, blockIdx.x, blockIdx.y, lds, red_lds,
                                                         a.red + (blockIdx.y * gridDim.x + blockIdx.x));
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
template <typename AT, int BLOCK, int KC, class POL, int QUANT, bool KAHAN>
static hipError_t launch(const StripArgs &a, hipStream_t s)
{
    const int Wt = BLOCK - 2 * a.rh;
    if (Wt < 1) return hipErrorInvalidValue;
    dim3 grid((a.io.W + Wt - 1) / Wt, (a.io.H + a.S - 1) / a.S);
    hipLaunchKernelGGL((strip_kernel<AT, BLOCK, KC, POL, QUANT, KAHAN>), grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// Orders per pass: the two LDS row buffers hold 2 * NCH * KC * (BLOCK + 1)
// elements, kept near 128 KiB of the 160 KiB per compute unit.
constexpr int kc_f32_fwd(int block) { return block == 256 ? 16 : block == 512 ? 8 : 4; }
constexpr int kc_f64_fwd(int block) { return block == 256 ? 8 : block == 512 ? 4 : 2; }
constexpr int kc_f32_train(int block) { return block == 256 ? 10 : block == 512 ? 5 : 2; }

int chunk_forward_f32(int block) { return kc_f32_fwd(block); }
int chunk_forward_f64(int block) { return kc_f64_fwd(block); }
int chunk_train_f32(int block) { return kc_f32_train(block); }
int chunk_backward_f32(int block) { return kc_f32_fwd(block); }
int acc_count_forward() { return PolForward<float>::NACC; }
int acc_count_train() { return PolTrain::NACC; }
int acc_count_backward() { return PolBackward::NACC; }

template <int QUANT, bool KAHAN>
static hipError_t fwd32(const StripArgs &a, int block, hipStream_t s)
{
    switch (block) {
    case 256: return launch<float, 256, kc_f32_fwd(256), PolForward<float>, QUANT, KAHAN>(a, s);
    case 512: return launch<float, 512, kc_f32_fwd(512), PolForward<float>, QUANT, KAHAN>(a, s);
    case 1024: return launch<float, 1024, kc_f32_fwd(1024), PolForward<float>, QUANT, KAHAN>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward_f32(const StripArgs &a, int block, int prec, int kahan, hipStream_t s)
{
    if (prec == 1) return kahan ? fwd32<1, true>(a, block, s) : fwd32<1, false>(a, block, s);
    if (prec == 2) return kahan ? fwd32<2, true>(a, block, s) : fwd32<2, false>(a, block, s);
    if (prec == 4) return kahan ? fwd32<4, true>(a, block, s) : fwd32<4, false>(a, block, s);
    return kahan ? fwd32<0, true>(a, block, s) : fwd32<0, false>(a, block, s);
}

hipError_t launch_forward_f64(const StripArgs &a, int block, hipStream_t s)
{
    switch (block) {
    case 256: return launch<double, 256, kc_f64_fwd(256), PolForward<double>, 0, false>(a, s);
    case 512: return launch<double, 512, kc_f64_fwd(512), PolForward<double>, 0, false>(a, s);
    case 1024: return launch<double, 1024, kc_f64_fwd(1024), PolForward<double>, 0, false>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_train_f32(const StripArgs &a, int block, hipStream_t s)
{
    switch (block) {
    case 256: return launch<float, 256, kc_f32_train(256), PolTrain, 0, false>(a, s);
    case 512: return launch<float, 512, kc_f32_train(512), PolTrain, 0, false>(a, s);
    case 1024: return launch<float, 1024, kc_f32_train(1024), PolTrain, 0, false>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int BLOCK>
static hipError_t bwd(const StripArgs &a, hipStream_t s)
{
    const int Wt = BLOCK - 2 * a.rh;
    if (Wt < 1) return hipErrorInvalidValue;
    dim3 grid((a.io.W + Wt - 1) / Wt, (a.io.H + a.S - 1) / a.S);
    hipLaunchKernelGGL((backward_kernel<BLOCK, kc_f32_fwd(BLOCK)>), grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_backward_f32(const StripArgs &a, int block, float *grad_sigma, double inv_sigma, int nred,
                               hipStream_t s)
{
    hipError_t e;
    switch (block) {
    case 256: e = bwd<256>(a, s); break;
    case 512: e = bwd<512>(a, s); break;
    case 1024: e = bwd<1024>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (grad_sigma) {
        hipLaunchKernelGGL(sigma_reduce_kernel, dim3(1), dim3(256), 0, s, nullptr, (const double *)a.red, nred,
                           inv_sigma, grad_sigma);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace bsk
