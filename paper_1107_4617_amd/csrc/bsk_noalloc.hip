// Allocation-free variant of the single-image forward: the partial
// accumulators of a multi-pass launch live in a fixed device array of this
// library instead of the per-stream workspace, so the call makes no device
// allocation at all (for callers under HIP graph capture or in loops where
// hipMalloc is not allowed).  The kernels are those of bilateral_shiftable_ex.
#include <cstring>
#include <mutex>

#include "bsk_host.h"

namespace {

// Scratch for the multi-pass accumulator planes: two FP32 planes of a
// 4096 x 4096 image (one FP64 plane pair of 4096 x 2048).  Every device the
// library runs on holds its own copy until the process ends.
constexpr size_t kScratchBytes = 128ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device.  In host code the array's name only
// stands for the symbol; its device address comes from hipGetSymbolAddress,
// taken once per device with that device current.
constexpr int kMaxDev = 64;
std::mutex g_mu;
void *g_ptr[kMaxDev] = {};

int scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bsk::host::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDev) return bsk::host::fail(BSK_EUNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return bsk::host::hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return BSK_OK;
}

}  // namespace

using namespace bsk::host;

extern "C" {

int bilateral_shiftable_noalloc(const void *img, int H, int W, int radius, float sigma_r, float T, void *out,
                                const bsk_options *opt, void *stream)
{
    if (!img || !out) return fail(BSK_EINVAL, "null image pointer");
    Resolved r;
    int st = resolve(H, W, radius, sigma_r, T, opt, &r, kForward);
    if (st) return st;
    if (r.range_kernel != BSK_RANGE_COS || r.sp.Ns > 0)
        return fail(BSK_EUNSUPPORTED, "the allocation-free forward runs the raised cosine with the box window");
    const size_t esz = r.prec == BSK_FP64 ? 8 : 4;
    if (overlap(img, ((size_t)(H - 1) * r.pitch_in + W) * esz, out, ((size_t)(H - 1) * r.pitch_out + W) * esz))
        return fail(BSK_EINVAL, "img and out overlap");
    const size_t need = r.plan.K > r.kc ? (size_t)bsk::acc_count_forward() * H * W * esz : 0;
    if (need > kScratchBytes)
        return fail(BSK_ENOMEM, "%d passes over %dx%d need %zu bytes of accumulators; the fixed scratch "
                    "holds %zu", (r.plan.K + r.kc - 1) / r.kc, H, W, need, kScratchBytes);
    void *p = nullptr;
    st = scratch_ptr(&p);
    if (st) return st;
    bsk::StripArgs a;
    fill_args(&a, r, H, W, r.kc);
    a.io.img = img;
    a.io.out = out;
    if (need > 0) a.ws = p;
    const hipError_t e = r.prec == BSK_FP64
                             ? bsk::launch_forward_f64(a, r.block, r.kc, (hipStream_t)stream)
                             : bsk::launch_forward_f32(a, r.block, r.kc, r.prec, r.kahan, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return BSK_OK;
}

}  // extern "C"
