// Persistent batched kernel: many images of different sizes, radii and
// sigma_r in one launch.  Each workgroup repeatedly claims a work unit
// (image, strip, row segment) from device counters and runs the same fused
// strip body as the single-image forward kernel on it; the loop ends for
// every workgroup once every queue's counter has passed its last unit, so the
// grid always drains.  Units are numbered image by image in the order of the
// host table, which lists the most expensive images first, and cut into one
// contiguous queue per XCD of about equal cost.
#include "bsk_device.h"

namespace bsk {

// Same pass shapes as the single-image FP32 forward (full pass).
constexpr int kc_batched(int block) { return block == 256 ? 16 : block == 512 ? 8 : 4; }
constexpr int kl_batched(int block) { return block == 256 ? 4 : block == 512 ? 2 : 1; }
// resident workgroups per compute unit: three 256-lane ones (LDS and
// registers), two of the wider ones
constexpr int wg_batched(int block) { return block == 256 ? 3 : 2; }
int wg_per_cu_batched(int block) { return wg_batched(block); }

int chunk_batched_f32(int block) { return kc_batched(block); }
// the 12-order pass of the 256-lane kernel (0: none), as for the single-image forward
constexpr int kmid_batched(int block) { return block == 256 ? 12 : 0; }
int mid_chunk_batched_f32(int block) { return kmid_batched(block); }
int max_radius_batched(int block) { return (block - 2) / 2; }

__global__ void reset_counter_kernel(unsigned *counter)
{
    if (threadIdx.x < kBatchQueues) counter[threadIdx.x] = 0u;
}

template <int BLOCK, int KC>
__global__ void __launch_bounds__(BLOCK, wg_batched(BLOCK)) batched_kernel(const BatchArgs a)
{
    __shared__ __align__(16) float lds[strip_lds_elems<PolForward<float>::NCH, kl_batched(BLOCK), BLOCK>()];
    __shared__ int unit_sh;
    // the XCD this workgroup runs on: workgroups are dispatched to the XCDs
    // round-robin by linear index
    const int home = blockIdx.x % kBatchQueues;
    for (;;) {
        if (threadIdx.x == 0) {
            // the home queue first, then the others in turn; -1 once all are empty
            int u = -1;
            for (int k = 0; k < kBatchQueues && u < 0; ++k) {
                const int q = (home + k) % kBatchQueues;
                const int len = a.qstart[q + 1] - a.qstart[q];
                if (len <= 0) continue;
                const int v = (int)atomicAdd(a.counter + q, 1u);
                if (v < len) u = a.qstart[q] + v;
            }
            unit_sh = u;
        }
        __syncthreads();
        const int unit = unit_sh;
        __syncthreads();
        if (unit < 0) break;
        // image owning this unit: last entry with unit0 <= unit
        int lo = 0, hi = a.nimg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.imgs[mid].unit0 <= unit) lo = mid;
            else hi = mid - 1;
        }
        const BatchImage im = a.imgs[lo];
        const int local = unit - im.unit0;
        const int bx = local % im.strips;
        const int by = local / im.strips;
        IO io;
        io.img = im.img;
        io.aux0 = io.aux1 = io.aux2 = io.aux3 = io.aux4 = nullptr;
        io.out = im.out;
        io.out2 = nullptr;
        io.H = im.H;
        io.W = im.W;
        io.pitch_in = im.W;
        io.pitch_out = im.W;
        Geom gm;
        gm.H = im.H;
        gm.W = im.W;
        gm.pitch_in = im.W;
        gm.pitch_out = im.W;
        gm.rh = im.rh;
        gm.rv = im.rv;
        gm.S = im.S;
        gm.K = im.K;
        gm.start_mode = im.start_mode;
        gm.omega_base = im.omega_base;
        gm.delta = im.delta;
        gm.v = a.vtab + im.v_off;
        gm.vf = a.vtabf + im.v_off;
        gm.ws = im.ws_off >= 0 ? (void *)(a.ws + im.ws_off) : nullptr;
        gm.sp_u0 = 1.0f;   // the box spatial kernel
        for (int j = 0; j < kMaxSpatialFreq; ++j) gm.sp_u[j] = 0.0f;
        gm.sp_row = gm.sp_col = nullptr;
        // the image's pass size: the full pass, its half or (256 lanes) 12 orders (same LDS shape)
        constexpr int KM = kmid_batched(BLOCK);
        if (im.kc == KC)
            strip_body<float, BLOCK, KC, kl_batched(BLOCK), PolForward<float>, 0, false>(io, gm, bx, by, lds,
                                                                                        nullptr, nullptr);
        else if (KM > 0 && im.kc == KM)
            strip_body<float, BLOCK, (KM > 0 ? KM : KC), kl_batched(BLOCK), PolForward<float>, 0, false>(
                io, gm, bx, by, lds, nullptr, nullptr);
        else
            strip_body<float, BLOCK, KC / 2, kl_batched(BLOCK), PolForward<float>, 0, false>(io, gm, bx, by, lds,
                                                                                            nullptr, nullptr);
        __syncthreads();
    }
}

hipError_t launch_batched_f32(const BatchArgs &a, int block, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, a.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (block) {
    case 256: hipLaunchKernelGGL((batched_kernel<256, kc_batched(256)>), dim3(grid), dim3(256), 0, s, a); break;
    case 512: hipLaunchKernelGGL((batched_kernel<512, kc_batched(512)>), dim3(grid), dim3(512), 0, s, a); break;
    case 1024: hipLaunchKernelGGL((batched_kernel<1024, kc_batched(1024)>), dim3(grid), dim3(1024), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bsk
