// C ABI of libbsk: argument validation, planning, workspace and launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "bsk_host.h"

namespace bsk {
namespace host {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(BSK_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ----------------------------------------------------------- workspace --
// One grow-only device buffer per (device, stream, slot).  Calls that share a
// stream are ordered by it, so they may share the buffer.
struct WsKey {
    int dev;
    void *stream;
    int slot;
    bool operator<(const WsKey &o) const
    {
        if (dev != o.dev) return dev < o.dev;
        if (stream != o.stream) return stream < o.stream;
        return slot < o.slot;
    }
};
struct WsBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    unsigned long long gen = 0;
};
std::mutex g_ws_mu;
std::map<WsKey, WsBuf> g_ws;
unsigned long long g_ws_gen = 0;
long long g_ws_limit = 0;   // bytes of library workspace per device; 0 = unlimited

int get_ws(void *stream, int slot, size_t bytes, void **out, unsigned long long *gen)
{
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        if (g_ws_limit > 0 && bytes > (size_t)g_ws_limit)
            return fail(BSK_ENOMEM, "workspace of %zu bytes exceeds the limit of %lld bytes", bytes, g_ws_limit);
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    WsBuf &b = g_ws[WsKey{dev, stream, slot}];
    if (b.bytes < bytes) {
        if (g_ws_limit > 0) {
            size_t held = 0;
            for (auto &kv : g_ws)
                if (kv.first.dev == dev) held += kv.second.bytes;
            if (held - b.bytes + bytes > (size_t)g_ws_limit)
                return fail(BSK_ENOMEM, "workspace of %zu bytes would exceed the limit of %lld bytes "
                            "(%zu held on the device)", bytes, g_ws_limit, held);
        }
        if (b.ptr) {
            // the previous buffer may still be read by queued work on this stream
            e = hipStreamSynchronize((hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        e = hipMalloc(&b.ptr, bytes);
        if (e != hipSuccess) {
            b.ptr = nullptr;
            (void)hipGetLastError();
            return fail(BSK_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
        }
        b.bytes = bytes;
        b.gen = ++g_ws_gen;
    }
    *out = b.ptr;
    if (gen) *gen = b.gen;
    return BSK_OK;
}

int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// ----------------------------------------------------------- validation --
bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Orders per pass from the pass sizes a kernel family offers (full and a
// smaller one, by default full / 2):
// the one with the lower estimated cost, counting the padded orders each pass
// runs and about 2.5 + kc / 10 orders' worth of per-pass work (window
// initialisation, recurrence starts, workspace traffic).
// padded orders plus a per-pass cost (window initialisation, three recurrence
// starts per row, workspace traffic) of about 5 + kc / 10 orders
static double chunk_cost(int K, int kc) { return ((K + kc - 1) / kc) * (kc + 5.0 + 0.1 * kc); }

int pick_chunk(int K, int full, int small, int mid)
{
    if (small == 0) small = full / 2;
    int best = full;
    if (small >= 1 && small != full && chunk_cost(K, small) < chunk_cost(K, best)) best = small;
    if (mid > 0 && chunk_cost(K, mid) < chunk_cost(K, best)) best = mid;
    return best;
}

int pick_chunk_of(int K, const int *sizes, int n)
{
    int best = sizes[0];
    for (int i = 1; i < n; ++i)
        if (chunk_cost(K, sizes[i]) < chunk_cost(K, best)) best = sizes[i];
    return best;
}

std::shared_ptr<const bsk::PolyPlan> poly_plan(int N, double sigma_r, double T, double eps)
{
    static std::mutex mu;
    static std::map<std::tuple<int, double, double, double>, std::shared_ptr<const bsk::PolyPlan>> cache;
    const auto key = std::make_tuple(N, sigma_r, T, eps);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    auto p = std::make_shared<bsk::PolyPlan>();
    if (bsk::make_poly_plan(N, sigma_r, T, eps, p.get()) != 0) return nullptr;
    if (cache.size() > 64) cache.clear();
    cache[key] = p;
    return p;
}

// Channel pairs per pass of the polynomial kernel: the full pass or its half,
// whichever has the lower estimated cost.  Per pixel a pass costs about 16
// VALU instructions per channel (transforms, sums, scan, recombination), 7 per
// step of the coefficient recurrence over its channels, 100 for its starts
// and, when there are several passes, the equivalent of about 250 for the
// workspace traffic (48 bytes per pixel); the first pass also runs the
// recurrence from d_2N down to its channels.
static int pick_chunk_poly(int pairs, int N, int full, int big)
{
    auto cost = [&](int kc) {
        const int np = (pairs + kc - 1) / kc * kc;
        const int passes = np / kc;
        double c = passes * (2.0 * kc * 16.0 + 7.0 * (2 * kc + 2) + 100.0 + (passes > 1 ? 250.0 : 0.0));
        c += 7.0 * std::max(0, 2 * N - 2 * np);
        return c;
    };
    int kc = cost(full / 2) < cost(full) ? full / 2 : full;
    if (big > 0 && cost(big) < cost(kc)) kc = big;
    return kc;
}

// Workgroups per compute unit of the kernel a resolved request will launch.
static int kernel_occupancy(const Resolved &r, int kind)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int, int, int, int>, int> cache;
    // the radius picks the compile-time-radius kernels where they exist, and
    // the padded order count and start mode their one-pass forms, whose
    // register counts (and so residency) differ from the other kernels'
    const bool cosine = kind != kPatch2 && r.range_kernel != BSK_RANGE_POLY;
    const int Kpad = cosine && r.kc > 0 ? (r.plan.K + r.kc - 1) / r.kc * r.kc : 0;
    const int smode = cosine ? r.plan.start_mode : 0;
    const auto key = std::make_tuple(kind + 3 * r.range_kernel, r.block, r.kc, r.prec, r.kahan,
                                     r.sp.nsc * 2 + (r.sp.even ? 1 : 0), r.rh,
                                     Kpad <= r.kc ? smode : 2 + smode, [] {
        int d = 0;
        (void)hipGetDevice(&d);
        return d;
    }());
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    bsk::StripArgs a;
    std::memset(&a, 0, sizeof(a));
    a.rh = r.rh;
    a.K = Kpad;
    a.start_mode = smode;
    int occ = 1;
    if (kind == kPatch2) {
        (void)bsk::launch_patch2_f32(a, r.block, r.kc, 0, nullptr, &occ);
    } else if (r.range_kernel == BSK_RANGE_POLY) {
        bsk::PolyArgs pa;
        std::memset(&pa, 0, sizeof(pa));
        pa.rh = r.rh;
        if (r.prec == BSK_FP64) (void)bsk::launch_poly_f64(pa, r.block, nullptr, &occ);
        else (void)bsk::launch_poly_f32(pa, r.block, r.kc, nullptr, &occ);
    } else if (r.sp.Ns > 0) {
        (void)bsk::launch_spatial_f32(a, r.block, r.sp, r.kc, nullptr, &occ);
    } else if (kind == kTrain) {
        (void)bsk::launch_train_f32(a, r.block, r.kc, nullptr, &occ);
    } else if (kind == kBackward) {
        (void)bsk::launch_backward_f32(a, r.block, r.kc, nullptr, 0.0, 0, nullptr, &occ);
    } else if (r.prec == BSK_FP64) {
        (void)bsk::launch_forward_f64(a, r.block, r.kc, nullptr, &occ);
    } else {
        (void)bsk::launch_forward_f32(a, r.block, r.kc, r.prec, r.kahan, nullptr, &occ);
    }
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = occ;
    return occ;
}

int resolve(int H, int W, int radius, float sigma_r, float T, const bsk_options *opt, Resolved *r, int kind,
            int nimg)
{
    if (H < 1 || W < 1) return fail(BSK_EINVAL, "image size %dx%d must be positive", H, W);
    if (radius < 0) return fail(BSK_EINVAL, "radius %d must be >= 0", radius);
    if (!finite_pos(sigma_r)) return fail(BSK_EINVAL, "sigma_r must be finite and > 0");
    if (!finite_pos(T)) return fail(BSK_EINVAL, "T must be finite and > 0");
    bsk_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    if (o.order_mode != 0 && o.order_mode != 1) return fail(BSK_EINVAL, "order_mode must be 0 or 1");
    if (o.order_mode == 1 && o.N < 0) return fail(BSK_EINVAL, "N must be >= 0");
    if (o.precision < BSK_FP32 || o.precision > BSK_I16) return fail(BSK_EINVAL, "unknown precision");
    if (!(o.weight_eps >= 0.0) || !std::isfinite(o.weight_eps))
        return fail(BSK_EINVAL, "weight_eps must be finite and >= 0");
    if (o.pitch_in < 0 || o.pitch_out < 0) return fail(BSK_EINVAL, "pitches must be >= 0");
    r->pitch_in = o.pitch_in ? o.pitch_in : W;
    r->pitch_out = o.pitch_out ? o.pitch_out : W;
    if (r->pitch_in < W || r->pitch_out < W) return fail(BSK_EINVAL, "pitch smaller than W");
    r->prec = o.precision;
    r->kahan = o.kahan ? 1 : 0;
    const long long nmax = (long long)H * (long long)W;
    if (nmax > (1LL << 40)) return fail(BSK_EINVAL, "image too large");

    if (o.range_kernel != BSK_RANGE_COS && o.range_kernel != BSK_RANGE_POLY)
        return fail(BSK_EINVAL, "unknown range_kernel %d", o.range_kernel);
    r->range_kernel = o.range_kernel;
    const bool poly = o.range_kernel == BSK_RANGE_POLY;
    r->poly.reset();
    r->poly_pairs = 0;
    if (kind == kPatch2) {
        if (poly || o.spatial_N != 0)
            return fail(BSK_EUNSUPPORTED, "the two-pixel patch uses the raised cosine and the box window");
        if (r->prec != BSK_FP32 || r->kahan)
            return fail(BSK_EUNSUPPORTED, "the two-pixel patch runs in plain FP32");
    }
    if (poly) {
        if (kind != kForward) return fail(BSK_EUNSUPPORTED, "the polynomial range kernel has the forward filter only");
        if (o.spatial_N != 0) return fail(BSK_EUNSUPPORTED, "the polynomial range kernel uses the box spatial kernel");
        if ((r->prec != BSK_FP32 && r->prec != BSK_FP64) || r->kahan)
            return fail(BSK_EUNSUPPORTED, "the polynomial range kernel runs in FP32 or FP64 without compensation");
        if (o.order_mode == 1) {
            r->N = o.N;
        } else {
            const double x = (double)T / (double)sigma_r;
            if (!(0.5 * x * x <= (double)bsk::kMaxPolyOrder))
                return fail(BSK_ERANGE, "automatic polynomial order exceeds %d", bsk::kMaxPolyOrder);
            r->N = bsk::poly_order_for(sigma_r, T);
        }
        if (r->N > bsk::kMaxPolyOrder)
            return fail(BSK_ERANGE, "polynomial order N=%d exceeds %d", r->N, bsk::kMaxPolyOrder);
        r->poly = poly_plan(r->N, sigma_r, T, o.weight_eps);
        if (!r->poly) return fail(BSK_EINVAL, "bad polynomial kernel plan");
        r->poly_pairs = (r->poly->K + 2) / 2;
        r->plan = bsk::Plan();
    } else {
        if (o.order_mode == 1) {
            r->N = o.N;
        } else {
            const double x = 2.0 * (double)T / (M_PI * (double)sigma_r);
            if (!(x * x < 1e7)) return fail(BSK_ERANGE, "automatic order N_0 too large");
            r->N = bsk::order_for(sigma_r, T);
        }
        if (r->N > 1000000) return fail(BSK_ERANGE, "order N=%d too large", r->N);
        if (bsk::make_plan(r->N, sigma_r, o.weight_eps, &r->plan) != 0)
            return fail(BSK_ERANGE, "order N=%d leaves more than %d folded orders (raise weight_eps)", r->N,
                        bsk::kMaxOrders);
        if (r->plan.K == 0) return fail(BSK_EINVAL, "weight_eps %g drops every order of N=%d", o.weight_eps, r->N);
    }

    // Clamping the radius to the image leaves every truncated window unchanged
    // (offsets beyond the image never occur, so no spatial weight changes).
    r->rh = radius < W - 1 ? radius : W - 1;
    r->rv = radius < H - 1 ? radius : H - 1;
    if (r->rh > BSK_MAX_RADIUS)
        return fail(BSK_EUNSUPPORTED, "clamped radius %d exceeds %d", r->rh, BSK_MAX_RADIUS);

    // spatial kernel: order Ns (or N_0 for the window), its folded plan
    r->sp = bsk::SpatialPlan();
    if (o.spatial_N < -1) return fail(BSK_EINVAL, "spatial_N must be >= -1");
    if (o.spatial_N != 0) {
        if (!finite_pos(o.spatial_sigma)) return fail(BSK_EINVAL, "spatial_sigma must be finite and > 0");
        int Ns = o.spatial_N;
        if (Ns < 0) {
            const double x = 2.0 * (double)radius / (M_PI * o.spatial_sigma);
            if (!(x * x < 1e6)) return fail(BSK_ERANGE, "automatic spatial order too large");
            Ns = std::max(1, (int)std::ceil(x * x));
        }
        if (Ns > 2 * bsk::kMaxSpatialFreq)
            return fail(BSK_ERANGE, "spatial order %d exceeds %d (raise spatial_sigma)", Ns, 2 * bsk::kMaxSpatialFreq);
        if (bsk::make_spatial_plan(Ns, o.spatial_sigma, &r->sp) != 0)
            return fail(BSK_EINVAL, "bad spatial kernel");
        if (kind != kForward || r->prec != BSK_FP32 || r->kahan)
            return fail(BSK_EUNSUPPORTED, "the spatial kernel runs in the plain FP32 forward only");
    }
    const bool spatial = r->sp.Ns > 0;

    int block = o.block;
    int tuned_S = 0, tuned_kc = 0;
    if (kind == kForward && !spatial && !poly && o.block == 0 && o.strip_h == 0 && o.order_chunk == 0) {
        int tb = 0, ts = 0, tk = 0;
        if (tuned_shape(r->rh, r->plan.K, H, W, r->prec, &tb, &ts, &tk)) {
            block = tb;
            tuned_S = ts;
            tuned_kc = tk;
        }
    }
    if (block == 0) {
        block = 1024;
        const int cands[3] = {256, 512, 1024};
        for (int b : cands) {
            if (b - 2 * r->rh >= b / 2) {
                block = b;
                break;
            }
        }
    }
    if (block != 256 && block != 512 && block != 1024)
        return fail(BSK_EINVAL, "block must be 256, 512 or 1024");
    if (spatial && !bsk::spatial_block_ok(block, r->sp.nsc)) {
        if (o.block || !bsk::spatial_block_ok(512, r->sp.nsc) || 512 - 2 * r->rh < 1)
            return fail(BSK_EUNSUPPORTED, "spatial order %d with radius %d: no strip shape (256 lanes, or 512 "
                        "for orders up to 4)", r->sp.Ns, r->rh);
        block = 512;
    }
    if (block - 2 * r->rh < 1)
        return fail(BSK_EUNSUPPORTED, "radius %d too large for a %d-lane strip", r->rh, block);
    r->block = block;
    if (o.order_chunk < 0) return fail(BSK_EINVAL, "order_chunk must be >= 0");
    int kc = o.order_chunk ? o.order_chunk : tuned_kc;
    if (poly) {
        if (r->prec == BSK_FP64) {
            kc = bsk::chunk_poly_f64(block);
        } else {
            const int full = bsk::chunk_poly_f32(block);
            const int big = bsk::big_chunk_poly_f32(block, r->rh);
            if (o.order_chunk) {
                if (o.order_chunk != full && o.order_chunk != full / 2 && !(big && o.order_chunk == big))
                    return fail(BSK_EINVAL, "order_chunk %d is not a polynomial-kernel pass size (%d or %d%s)",
                                o.order_chunk, full, full / 2, big ? ", or 24 at this radius" : "");
                kc = o.order_chunk;
            } else {
                kc = pick_chunk_poly(r->poly_pairs, r->N, full, big);
            }
        }
    } else if (spatial) {
        const int full = bsk::chunk_spatial_f32(block, r->sp.nsc);
        const int small = bsk::chunk_spatial_small_f32(block, r->sp.nsc);
        if (o.order_chunk) {
            if (o.order_chunk != full && o.order_chunk != small)
                return fail(BSK_EINVAL, "order_chunk %d is not a spatial pass size (%d or %d)", o.order_chunk, full,
                            small);
            kc = o.order_chunk;
        } else {
            kc = pick_chunk(r->plan.K, full, small);
        }
    } else if (kind == kPatch2) {
        // the caller picks between the two pass sizes; residency is the same
        if (kc == 0) kc = bsk::chunk_forward_f32(block);
        if (!bsk::valid_chunk_forward_f32(block, kc))
            return fail(BSK_EINVAL, "order_chunk %d is not a pass size of a %d-lane block", kc, block);
    } else if (kind == kTrain) {
        kc = bsk::chunk_train_f32(block);
    } else if (kind == kBackward) {
        const int full = bsk::chunk_backward_f32(block), mid = bsk::mid_chunk_backward_f32(block);
        const int big = bsk::big_chunk_backward_f32(block);
        if (kc == 0) {
            // Measured per padded order (256 lanes, 4096^2 and 16 x 1024^2): the full
            // pass at two workgroups per CU costs 1, the 12-order pass 1.38 and the
            // half pass 1.55 (both at three per CU), so the full pass wins unless the
            // half pass saves a whole pass of it.  The 24-order pass (two per CU)
            // costs 0.93 (one pass of 24 against two of 16 on 22 orders).
            auto cost = [&](int c, double w) { return (double)((r->plan.K + c - 1) / c) * c * w; };
            kc = full;
            double best = cost(full, 1.0);
            if (mid && cost(mid, 1.38) < best) kc = mid, best = cost(mid, 1.38);
            if (cost(full / 2, 1.55) < best) kc = full / 2, best = cost(full / 2, 1.55);
            if (big && cost(big, 0.93) < best) kc = big, best = cost(big, 0.93);
        }
        if (!bsk::valid_chunk_backward_f32(block, kc) && !(mid && kc == mid) && !(big && kc == big))
            return fail(BSK_EINVAL, "order_chunk %d is not a pass size of a %d-lane block", kc, block);
    } else if (r->prec == BSK_FP64) {
        // one pass of up to 16 orders with the start mode as a constant where the
        // plan allows it, else passes of the general kernel
        const int one = bsk::onepass_chunk_forward_f64(block);
        kc = (one && r->plan.K <= one && r->plan.start_mode <= 1) ? one : bsk::chunk_forward_f64(block);
    } else {
        // the plain FP32 stack at 256 lanes has 8, 12 and 16 orders per pass (and
        // 20 and 24 at the compile-time radii), the others the full and the half pass
        int sizes[bsk::kMaxForwardChunks];
        const int n = bsk::forward_chunks_f32(block, r->prec, r->kahan, r->rh, sizes);
        if (kc == 0) kc = pick_chunk_of(r->plan.K, sizes, n);
        if (!bsk::forward_chunk_ok_f32(block, r->prec, r->kahan, r->rh, kc))
            return fail(BSK_EINVAL, "order_chunk %d is not a pass size of a %d-lane block", kc, block);
    }
    r->kc = kc;
    if (o.strip_h < 0) return fail(BSK_EINVAL, "strip_h must be >= 0");
    const int Wt = block - 2 * r->rh;
    const int strips = (W + Wt - 1) / Wt;
    if (o.strip_h > 0) {
        r->S = o.strip_h;
    } else if (tuned_S > 0) {
        r->S = tuned_S;
    } else {
        // Rows per workgroup: one round of resident workgroups of the kernel
        // that will run, so the 2 rv rows of window initialisation repeat as
        // seldom as the chip allows while every compute unit holds its full
        // complement.  (With the per-stage wave priorities of the strip body
        // one round beats two by 3-5% on every strip kernel.)  The segment
        // count rounds down, so a last, partial round of workgroups never
        // appears.
        const int bpc = kernel_occupancy(*r, kind);
        const long long target = 1LL * bpc * device_cus();
        long long segs = target / ((long long)strips * (nimg > 1 ? nimg : 1));
        if (segs < 1) segs = 1;
        int bestS = (int)((H + segs - 1) / segs);
        if (bestS < 8) bestS = 8;
        r->S = bestS;
    }
    if (r->S > H) r->S = H;
    return BSK_OK;
}

void fill_args(bsk::StripArgs *a, const Resolved &r, int H, int W, int kc)
{
    std::memset(a, 0, sizeof(*a));
    a->io.H = H;
    a->io.W = W;
    a->io.pitch_in = r.pitch_in;
    a->io.pitch_out = r.pitch_out;
    a->rh = r.rh;
    a->rv = r.rv;
    a->S = r.S;
    a->K = (r.plan.K + kc - 1) / kc * kc;
    a->omega_base = r.plan.omega_base;
    a->delta = r.plan.delta;
    a->start_mode = r.plan.start_mode;
    const int Wt = r.block - 2 * r.rh;
    a->strips = (W + Wt - 1) / Wt;
    for (int m = 0; m < a->K; ++m) {
        a->v[m] = m < r.plan.K ? r.plan.v[m] : 0.0;
        a->vf[m] = (float)a->v[m];
    }
}

int nblocks(const Resolved &r, int H, int W)
{
    const int Wt = r.block - 2 * r.rh;
    return ((W + Wt - 1) / Wt) * ((H + r.S - 1) / r.S);
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace host
}  // namespace bsk

using namespace bsk::host;

namespace {

// Coefficient tables of the polynomial kernel, uploaded to a workspace slot
// of the stream when the plan or the buffer changes.
struct PolyUpload {
    const bsk::PolyPlan *plan = nullptr;
    std::shared_ptr<const bsk::PolyPlan> keep;   // keeps the plan (and so the key) alive
    int np = 0;
    int prec = -1;
    unsigned long long gen = 0;   // workspace generation the table was uploaded into
    std::vector<unsigned char> host;
};
std::mutex g_poly_mu;
std::map<std::pair<int, void *>, PolyUpload> g_poly_up;

int poly_forward(const void *img, int H, int W, const Resolved &r, void *out, void *stream)
{
    const bsk::PolyPlan &pp = *r.poly;
    const int kc = r.kc;
    const int np = (r.poly_pairs + kc - 1) / kc * kc;
    const bool f64 = r.prec == BSK_FP64;
    const size_t esz = f64 ? 8 : 4;
    const size_t nrows = (size_t)(2 * std::max(pp.N, np) + 3) * bsk::kPolyRow;
    const size_t nsig = (size_t)(2 * np + 2);
    void *tab = nullptr;
    unsigned long long gen = 0;
    int st = get_ws(stream, kWsPolyTab, (nrows + nsig) * esz, &tab, &gen);
    if (st) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    {
        std::lock_guard<std::mutex> lk(g_poly_mu);
        PolyUpload &u = g_poly_up[std::make_pair(dev, stream)];
        if (u.plan != &pp || u.np != np || u.prec != r.prec || u.gen != gen) {
            if (!u.host.empty()) {
                // an earlier upload from the host copy may still be pending on the stream
                e = hipStreamSynchronize((hipStream_t)stream);
                if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            }
            u.host.assign((nrows + nsig) * esz, 0);
            auto put = [&](size_t i, double v) {
                if (f64) ((double *)u.host.data())[i] = v;
                else ((float *)u.host.data())[i] = (float)v;
            };
            for (size_t i = 0; i < pp.rows.size(); ++i) put(i, pp.rows[i]);
            // rows above the start shift the window by four
            for (size_t i = pp.rows.size(); i < nrows; i += bsk::kPolyRow) put(i + 4, 1.0);
            // sig[0] belongs to e_{-1}, which is zero
            for (size_t q = 1; q < nsig; ++q)
                put(nrows + q, (int)q - 1 < pp.K ? std::exp(pp.lsig[q - 1] - pp.lsig[0]) : 0.0);
            e = hipMemcpyAsync(tab, u.host.data(), u.host.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "coefficient table upload");
            u.plan = &pp;
            u.keep = r.poly;
            u.np = np;
            u.prec = r.prec;
            u.gen = gen;
        }
    }
    bsk::PolyArgs a;
    std::memset(&a, 0, sizeof(a));
    a.io.img = img;
    a.io.out = out;
    a.io.H = H;
    a.io.W = W;
    a.io.pitch_in = r.pitch_in;
    a.io.pitch_out = r.pitch_out;
    a.rh = r.rh;
    a.rv = r.rv;
    a.S = r.S;
    a.NP = np;
    a.N = pp.N;
    a.rho = pp.rho;
    a.inv_rho = 1.0 / pp.rho;
    a.rows = tab;
    a.sig = (const char *)tab + nrows * esz;
    if (np > kc) {
        void *ws = nullptr;
        st = get_ws(stream, kWsAcc, 6 * (size_t)H * W * esz, &ws);
        if (st) return st;
        a.ws = ws;
    }
    e = f64 ? bsk::launch_poly_f64(a, r.block, (hipStream_t)stream)
            : bsk::launch_poly_f32(a, r.block, kc, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "polynomial-kernel launch");
    return BSK_OK;
}

// Small per-call tables (the two-pixel patch's weights), uploaded to a
// workspace slot of the stream when their contents or the buffer change.
struct TabUpload {
    std::vector<unsigned char> host;
    unsigned long long gen = 0;   // workspace generation the table was uploaded into
};
std::mutex g_tab_mu;
std::map<std::tuple<int, void *, int>, TabUpload> g_tab_up;

int upload_table(void *stream, int slot, const std::vector<unsigned char> &bytes, void **out)
{
    void *dst = nullptr;
    unsigned long long gen = 0;
    int st = get_ws(stream, slot, bytes.size(), &dst, &gen);
    if (st) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_tab_mu);
    TabUpload &u = g_tab_up[std::make_tuple(dev, stream, slot)];
    if (u.gen != gen || u.host != bytes) {
        if (!u.host.empty()) {
            // an earlier upload from the host copy may still be pending on the stream
            e = hipStreamSynchronize((hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        }
        u.host = bytes;
        e = hipMemcpyAsync(dst, u.host.data(), u.host.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "table upload");
        u.gen = gen;
    }
    *out = dst;
    return BSK_OK;
}

int nlm2_impl(const float *img, int H, int W, int radius, float sigma_1, float sigma_2, int N1, int N2, int uy,
              int ux, float T, float *out, const bsk_options *opt, void *stream)
{
    if (!img || !out) return fail(BSK_EINVAL, "null image pointer");
    if (!finite_pos(sigma_2)) return fail(BSK_EINVAL, "sigma_2 must be finite and > 0");
    if (!finite_pos(sigma_1) || !finite_pos(T)) return fail(BSK_EINVAL, "sigma_1 and T must be finite and > 0");
    bsk_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    if (o.order_mode != 0) return fail(BSK_EINVAL, "the orders of the two-pixel patch are the N1 and N2 arguments");
    auto order = [&](int N, float sigma, int *res) -> int {
        if (N >= 0) {
            *res = N;
        } else {
            const double x = 2.0 * (double)T / (M_PI * (double)sigma);
            if (!(x * x < 1e6)) return fail(BSK_ERANGE, "automatic order too large");
            *res = bsk::order_for(sigma, T);
        }
        if (*res > 1000) return fail(BSK_ERANGE, "order %d exceeds 1000", *res);
        return BSK_OK;
    };
    int n1 = 0, n2 = 0;
    int st = order(N1, sigma_1, &n1);
    if (st) return st;
    st = order(N2, sigma_2, &n2);
    if (st) return st;
    // launch shape: the forward's rules at the first pixel's order
    bsk_options ro = o;
    ro.order_mode = 1;
    ro.N = n1;
    Resolved r;
    st = resolve(H, W, radius, sigma_1, T, &ro, &r, kPatch2);
    if (st) return st;
    if (overlap(img, ((size_t)(H - 1) * r.pitch_in + W) * 4, out, ((size_t)(H - 1) * r.pitch_out + W) * 4))
        return fail(BSK_EINVAL, "img and out overlap");

    // First pixel: the unfolded terms n of cos^N1 (frequency (2n - N1) / (sigma_1 sqrt N1),
    // weight 2^-N1 C(N1, n)) whose weight is at least eps, a contiguous range since
    // the weights are unimodal; second pixel: the folded plan of cos^N2.
    std::vector<double> w1;
    int nlo = 0;
    {
        double lw = -(double)n1 * std::log(2.0);   // log weight of n = 0
        for (int n = 0; n <= n1; ++n) {
            const double w = std::exp(lw);
            if (o.weight_eps <= 0.0 || w >= o.weight_eps) {
                if (w1.empty()) nlo = n;
                w1.push_back(w);
            }
            lw += std::log((double)(n1 - n)) - std::log((double)(n + 1));
        }
    }
    bsk::Plan p2;
    if (bsk::make_plan(n2, sigma_2, o.weight_eps, &p2) != 0)
        return fail(BSK_ERANGE, "order N2=%d leaves more than %d folded orders", n2, bsk::kMaxOrders);
    const int K1 = (int)w1.size(), K2 = p2.K;
    if (K1 == 0 || K2 == 0) return fail(BSK_EINVAL, "weight_eps %g drops every term", o.weight_eps);
    // Layout of the K1 x K2 terms over passes of kc orders.  Unpacked, each
    // first-pixel term spans ceil(K2 / kc) passes of its own.  Packed (256-lane
    // strips, 16-order passes, K2 <= 8), floor(16 / K2) whole terms share each
    // pass and the chains restart between them.
    const int full = bsk::chunk_forward_f32(r.block);
    auto unpacked = [&](int c) { return (long long)K1 * ((K2 + c - 1) / c); };
    auto cost = [&](long long np, int c) { return (double)np * (c + 2.5 + 0.1 * c); };
    const bool can_pack = r.block == 256 && full == bsk::kPatchPackPass && K2 <= bsk::kPatchPackMax;
    const int gpp = can_pack ? full / K2 : 0;
    const long long np_packed = can_pack ? (K1 + gpp - 1) / gpp : 0;
    int kc = r.kc, pack = 0;
    if (o.order_chunk == 0) {
        kc = cost(unpacked(full / 2), full / 2) < cost(unpacked(full), full) ? full / 2 : full;
        if (can_pack && cost(np_packed, full) <= cost(unpacked(kc), kc)) kc = full;
    }
    if (can_pack && kc == full) pack = K2;
    const int G2 = pack ? K2 : (K2 + kc - 1) / kc * kc;
    const long long K = pack ? np_packed * kc : (long long)K1 * G2;
    if (K > 65536) return fail(BSK_ERANGE, "%lld patch orders (raise weight_eps or the sigmas)", K);
    std::vector<unsigned char> tab((size_t)K * sizeof(float), 0);
    float *vf = (float *)tab.data();
    for (int g = 0; g < K1; ++g) {
        const size_t base = pack ? (size_t)(g / gpp) * kc + (size_t)(g % gpp) * K2 : (size_t)g * G2;
        for (int m = 0; m < K2; ++m) vf[base + m] = (float)(w1[g] * p2.v[m]);
    }
    void *dtab = nullptr;
    st = upload_table(stream, kWsPatchTab, tab, &dtab);
    if (st) return st;

    bsk::StripArgs a;
    std::memset(&a, 0, sizeof(a));
    a.io.img = img;
    a.io.out = out;
    a.io.H = H;
    a.io.W = W;
    a.io.pitch_in = r.pitch_in;
    a.io.pitch_out = r.pitch_out;
    a.io.uy = uy;
    a.io.ux = ux;
    a.rh = r.rh;
    a.rv = r.rv;
    a.S = r.S;
    a.K = (int)K;
    a.start_mode = 2;
    a.omega_base = p2.omega_base;
    a.delta = p2.delta;
    const int Wt = r.block - 2 * r.rh;
    a.strips = (W + Wt - 1) / Wt;
    a.p2_group = G2;
    const double s1 = n1 > 0 ? 1.0 / ((double)sigma_1 * std::sqrt((double)n1)) : 0.0;
    a.p2_omega1_base = (double)(2 * nlo - n1) * s1;
    a.p2_delta1 = 2.0 * s1;
    a.vf_dev = (const float *)dtab;
    if (K > kc) {
        void *ws = nullptr;
        st = get_ws(stream, kWsAcc, (size_t)bsk::acc_count_forward() * H * W * 4, &ws);
        if (st) return st;
        a.ws = ws;
    }
    hipError_t e = bsk::launch_patch2_f32(a, r.block, kc, pack, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "two-pixel-patch launch");
    return BSK_OK;
}

int forward_impl(const void *img, int H, int W, int radius, float sigma_r, float T, void *out,
                 const bsk_options *opt, void *stream)
{
    if (!img || !out) return fail(BSK_EINVAL, "null image pointer");
    Resolved r;
    int st = resolve(H, W, radius, sigma_r, T, opt, &r, kForward);
    if (st) return st;
    const size_t esz = r.prec == BSK_FP64 ? 8 : 4;
    if (overlap(img, ((size_t)(H - 1) * r.pitch_in + W) * esz, out, ((size_t)(H - 1) * r.pitch_out + W) * esz))
        return fail(BSK_EINVAL, "img and out overlap");
    if (r.range_kernel == BSK_RANGE_POLY) return poly_forward(img, H, W, r, out, stream);
    bsk::StripArgs a;
    const int kc = r.kc;
    fill_args(&a, r, H, W, kc);
    a.io.img = img;
    a.io.out = out;
    if (r.plan.K > kc) {
        void *ws = nullptr;
        st = get_ws(stream, kWsAcc, (size_t)bsk::acc_count_forward() * H * W * esz, &ws);
        if (st) return st;
        a.ws = ws;
    }
    if (r.sp.Ns > 0) {
        // phase tables (cos, sin)(nu_j y) for the rows and columns, then the kernel
        void *tab = nullptr;
        const size_t nrow = (size_t)H * r.sp.nsc * 2, ncol = (size_t)W * r.sp.nsc * 2;
        st = get_ws(stream, kWsPhase, (nrow + ncol) * sizeof(float), &tab);
        if (st) return st;
        float *rowtab = (float *)tab, *coltab = rowtab + nrow;
        hipError_t e = bsk::launch_phase_table(r.sp, H, rowtab, (hipStream_t)stream);
        if (e == hipSuccess) e = bsk::launch_phase_table(r.sp, W, coltab, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "phase table launch");
        a.sp_u0 = (float)r.sp.u0;
        for (int j = 0; j < bsk::kMaxSpatialFreq; ++j) a.sp_u[j] = (float)r.sp.u[j];
        a.sp_row = rowtab;
        a.sp_col = coltab;
        e = bsk::launch_spatial_f32(a, r.block, r.sp, r.kc, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "spatial forward launch");
        return BSK_OK;
    }
    hipError_t e = r.prec == BSK_FP64
                       ? bsk::launch_forward_f64(a, r.block, r.kc, (hipStream_t)stream)
                       : bsk::launch_forward_f32(a, r.block, r.kc, r.prec, r.kahan, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return BSK_OK;
}

// Training forward of B stacked images (B = 1: one image): img and out are
// [B][H][W], saved is [B][3][H][W].
int train_impl(const float *img, int B, int H, int W, const Resolved &r, float *out, float *saved, void *stream)
{
    bsk::StripArgs a;
    fill_args(&a, r, H, W, r.kc);
    a.io.img = img;
    a.io.out = out;
    a.io.out2 = saved;
    const long long plane = (long long)H * W * 4;
    a.nimg = B;
    a.bs_img = a.bs_out = plane;
    a.bs_out2 = 3 * plane;
    if (r.plan.K > r.kc) {
        void *ws = nullptr;
        int st = get_ws(stream, kWsTrainAcc, (size_t)bsk::acc_count_train() * plane * B, &ws);
        if (st) return st;
        a.ws = ws;
        a.bs_ws = bsk::acc_count_train() * plane;
    }
    hipError_t e = bsk::launch_train_f32(a, r.block, r.kc, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "train launch");
    return BSK_OK;
}

int train_entry(const float *img, int B, int H, int W, int radius, float sigma_r, float T, const bsk_options *opt,
                float *out, float *saved, void *stream)
{
    if (!img || !out || !saved) return fail(BSK_EINVAL, "null pointer");
    if (B < 1) return fail(BSK_EINVAL, "need at least one image");
    Resolved r;
    int st = resolve(H, W, radius, sigma_r, T, opt, &r, kTrain, B);
    if (st) return st;
    if (r.prec != BSK_FP32 || r.kahan)
        return fail(BSK_EUNSUPPORTED, "the training forward is FP32 without compensation");
    if (r.pitch_in != W || r.pitch_out != W) return fail(BSK_EUNSUPPORTED, "training forward needs dense pitch");
    const size_t n = (size_t)H * W * 4 * B;
    if (overlap(img, n, out, n) || overlap(img, n, saved, 3 * n) || overlap(out, n, saved, 3 * n))
        return fail(BSK_EINVAL, "buffers overlap");
    return train_impl(img, B, H, W, r, out, saved, stream);
}

int backward_entry(const float *img, const float *grad_out, const float *out, const float *saved, int B, int H, int W,
                   int radius, float sigma_r, float T, const bsk_options *opt, float *grad_img, float *grad_sigma,
                   void *stream)
{
    if (!img || !grad_out) return fail(BSK_EINVAL, "null pointer");
    if (B < 1) return fail(BSK_EINVAL, "need at least one image");
    if ((out == nullptr) != (saved == nullptr)) return fail(BSK_EINVAL, "out and saved must both be given or both NULL");
    Resolved r;
    int st = resolve(H, W, radius, sigma_r, T, opt, &r, kBackward, B);
    if (st) return st;
    if (r.prec != BSK_FP32 || r.kahan) return fail(BSK_EUNSUPPORTED, "the adjoint is FP32");
    if (r.pitch_in != W || r.pitch_out != W) return fail(BSK_EUNSUPPORTED, "the adjoint needs dense pitch");
    const size_t n = (size_t)H * W * 4 * B;
    if (grad_img && (overlap(grad_img, n, img, n) || overlap(grad_img, n, grad_out, n)))
        return fail(BSK_EINVAL, "grad_img overlaps an input");
    if (!grad_img && !grad_sigma) return BSK_OK;

    const long long plane = (long long)H * W * 4;
    if (!out) {
        void *tmp = nullptr;
        st = get_ws(stream, kWsBwdTrain, 4 * n, &tmp);
        if (st) return st;
        float *u = (float *)tmp;
        float *sv = u + (size_t)H * W * B;
        // the training forward with its own launch shape
        Resolved rt;
        st = resolve(H, W, radius, sigma_r, T, opt, &rt, kTrain, B);
        if (st) return st;
        st = train_impl(img, B, H, W, rt, u, sv, stream);
        if (st) return st;
        out = u;
        saved = sv;
    }
    bsk::StripArgs a;
    fill_args(&a, r, H, W, r.kc);
    a.io.img = img;
    a.io.aux0 = grad_out;
    a.io.aux1 = saved;                      // Q
    a.io.aux2 = out;                        // u
    a.io.aux3 = saved + (size_t)H * W;      // E1
    a.io.aux4 = saved + 2 * (size_t)H * W;  // E2
    a.io.out = grad_img;
    a.nimg = B;
    a.bs_img = plane;
    a.bs_out = grad_img ? plane : 0;
    a.bs_aux[0] = a.bs_aux[2] = plane;
    a.bs_aux[1] = a.bs_aux[3] = a.bs_aux[4] = 3 * plane;
    const int nred = nblocks(r, H, W) * B;
    void *red = nullptr;
    st = get_ws(stream, kWsBwdRed, (size_t)nred * sizeof(double), &red);
    if (st) return st;
    a.red = (double *)red;
    if (r.plan.K > r.kc) {
        void *ws = nullptr;
        st = get_ws(stream, kWsBwdAcc, (size_t)bsk::acc_count_backward() * plane * B, &ws);
        if (st) return st;
        a.ws = ws;
        a.bs_ws = bsk::acc_count_backward() * plane;
    }
    hipError_t e = bsk::launch_backward_f32(a, r.block, r.kc, grad_sigma, 1.0 / (double)sigma_r, nred,
                                            (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return BSK_OK;
}

}  // namespace

extern "C" {

int bilateral_shiftable(const float *img, int H, int W, int radius, float sigma_r, float T, float *out)
{
    int st = forward_impl(img, H, W, radius, sigma_r, T, out, nullptr, nullptr);
    if (st) return st;
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return BSK_OK;
}

int bilateral_shiftable_ex(const void *img, int H, int W, int radius, float sigma_r, float T, void *out,
                           const bsk_options *opt, void *stream)
{
    return forward_impl(img, H, W, radius, sigma_r, T, out, opt, stream);
}

int bilateral_shiftable_nlm2(const float *img, int H, int W, int radius, float sigma_1, float sigma_2, int N1,
                             int N2, int uy, int ux, float T, float *out, const bsk_options *opt, void *stream)
{
    return nlm2_impl(img, H, W, radius, sigma_1, sigma_2, N1, N2, uy, ux, T, out, opt, stream);
}

int bilateral_shiftable_train(const float *img, int H, int W, int radius, float sigma_r, float T,
                              const bsk_options *opt, float *out, float *saved, void *stream)
{
    return train_entry(img, 1, H, W, radius, sigma_r, T, opt, out, saved, stream);
}

int bilateral_shiftable_train_stack(const float *img, int B, int H, int W, int radius, float sigma_r, float T,
                                    const bsk_options *opt, float *out, float *saved, void *stream)
{
    return train_entry(img, B, H, W, radius, sigma_r, T, opt, out, saved, stream);
}

int bilateral_shiftable_backward(const float *img, const float *grad_out, const float *out, const float *saved,
                                 int H, int W, int radius, float sigma_r, float T, const bsk_options *opt,
                                 float *grad_img, float *grad_sigma, void *stream)
{
    return backward_entry(img, grad_out, out, saved, 1, H, W, radius, sigma_r, T, opt, grad_img, grad_sigma,
                          stream);
}

int bilateral_shiftable_backward_stack(const float *img, const float *grad_out, const float *out,
                                       const float *saved, int B, int H, int W, int radius, float sigma_r, float T,
                                       const bsk_options *opt, float *grad_img, float *grad_sigma, void *stream)
{
    return backward_entry(img, grad_out, out, saved, B, H, W, radius, sigma_r, T, opt, grad_img, grad_sigma,
                          stream);
}

int bsk_order_for(float sigma_r, float T)
{
    if (!finite_pos(sigma_r) || !finite_pos(T)) return fail(-1, "sigma_r and T must be finite and > 0");
    const double x = 2.0 * (double)T / (M_PI * (double)sigma_r);
    if (!(x * x < 2e9)) return fail(-1, "order too large");
    return bsk::order_for(sigma_r, T);
}

int bsk_plan_info(int N, double eps, int *K, double *dropped)
{
    if (N < 0 || N > 1000000) return fail(BSK_EINVAL, "N out of range");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BSK_EINVAL, "eps must be finite and >= 0");
    bsk::plan_counts(N, eps, K, dropped);
    return BSK_OK;
}

double bsk_truncation_error(int N, double eps)
{
    double d = 0.0;
    if (bsk_plan_info(N, eps, nullptr, &d) != BSK_OK) return -1.0;
    return d;
}

int bsk_poly_order_for(float sigma_r, float T)
{
    if (!finite_pos(sigma_r) || !finite_pos(T)) return fail(-1, "sigma_r and T must be finite and > 0");
    const double x = (double)T / (double)sigma_r;
    if (!(0.5 * x * x < 2e9)) return fail(-1, "order too large");
    return bsk::poly_order_for(sigma_r, T);
}

int bsk_poly_plan_info(int N, float sigma_r, float T, double eps, int *coefs, double *bound)
{
    if (!finite_pos(sigma_r) || !finite_pos(T)) return fail(BSK_EINVAL, "sigma_r and T must be finite and > 0");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BSK_EINVAL, "eps must be finite and >= 0");
    if (N < 0) {
        const double x = (double)T / (double)sigma_r;
        if (!(0.5 * x * x <= (double)bsk::kMaxPolyOrder))
            return fail(BSK_ERANGE, "automatic polynomial order exceeds %d", bsk::kMaxPolyOrder);
        N = bsk::poly_order_for(sigma_r, T);
    }
    if (N > bsk::kMaxPolyOrder) return fail(BSK_ERANGE, "polynomial order N=%d exceeds %d", N, bsk::kMaxPolyOrder);
    auto p = poly_plan(N, sigma_r, T, eps);
    if (!p) return fail(BSK_EINVAL, "bad polynomial kernel plan");
    if (coefs) *coefs = p->K;
    if (bound) *bound = p->bound;
    return BSK_OK;
}

const char *bsk_last_error(void) { return g_err; }

int bsk_set_workspace_limit(long long bytes)
{
    if (bytes < 0) return fail(BSK_EINVAL, "workspace limit must be >= 0");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    g_ws_limit = bytes;
    return BSK_OK;
}

void bsk_release_batched(void);

int bsk_release(void)
{
    bsk_release_batched();
    std::lock_guard<std::mutex> lk(g_ws_mu);
    hipError_t e = hipDeviceSynchronize();
    for (auto &kv : g_ws) {
        if (kv.second.ptr) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(kv.first.dev);
            (void)hipFree(kv.second.ptr);
            (void)hipSetDevice(cur);
        }
    }
    g_ws.clear();
    {
        std::lock_guard<std::mutex> lp(g_poly_mu);
        g_poly_up.clear();
    }
    {
        std::lock_guard<std::mutex> lt(g_tab_mu);
        g_tab_up.clear();
    }
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    return BSK_OK;
}

const char *bsk_version(void) { return "bsk 0.1 (gfx950)"; }

}  // extern "C"

// Batched entry points and the autotuner are implemented in bsk_batched.cpp.
