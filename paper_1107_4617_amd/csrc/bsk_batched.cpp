// Batched entry points (one persistent launch, optionally replayed from a HIP
// graph) and the launch-shape autotuner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "bsk_host.h"

using namespace bsk::host;

namespace {

// --------------------------------------------------------------- tables --
struct BatchPlan {
    std::vector<bsk::BatchImage> imgs;
    std::vector<double> vtab;
    std::vector<float> vtabf;
    long long ws_elems = 0;
    int total_units = 0;
    int block = 256;
};

constexpr int kBatchRows = 96;   // default output rows per work unit (64: 1% slower on the 256-image batch)

int build_batch(const bsk_image_desc *d, int B, float T, const bsk_options *opt, BatchPlan *bp)
{
    if (!d || B < 1) return fail(BSK_EINVAL, "need at least one descriptor");
    if (!finite_pos(T)) return fail(BSK_EINVAL, "T must be finite and > 0");
    bsk_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    if (o.precision != BSK_FP32 || o.kahan) return fail(BSK_EUNSUPPORTED, "the batched path is FP32");
    if (o.spatial_N != 0) return fail(BSK_EUNSUPPORTED, "the batched path uses the box spatial kernel");
    if (o.range_kernel != BSK_RANGE_COS) return fail(BSK_EUNSUPPORTED, "the batched path uses the raised cosine");
    if (o.pitch_in || o.pitch_out) return fail(BSK_EUNSUPPORTED, "the batched path needs dense pitch");
    if (o.strip_h < 0 || !(o.weight_eps >= 0.0)) return fail(BSK_EINVAL, "bad options");

    struct Item {
        bsk::BatchImage im;
        std::vector<double> v;
        double cost;
    };
    std::vector<Item> items;
    items.reserve(B);
    int max_rh = 0;
    for (int b = 0; b < B; ++b) {
        const bsk_image_desc &q = d[b];
        if (!q.img || !q.out) return fail(BSK_EINVAL, "descriptor %d: null pointer", b);
        if (q.H < 1 || q.W < 1 || q.radius < 0) return fail(BSK_EINVAL, "descriptor %d: bad size or radius", b);
        if (!finite_pos(q.sigma_r)) return fail(BSK_EINVAL, "descriptor %d: sigma_r must be finite and > 0", b);
        const size_t n = (size_t)q.H * q.W * 4;
        if (overlap(q.img, n, q.out, n)) return fail(BSK_EINVAL, "descriptor %d: img and out overlap", b);
        int N = q.N;
        if (N < 0) {
            const double x = 2.0 * (double)T / (M_PI * (double)q.sigma_r);
            if (!(x * x < 1e7)) return fail(BSK_ERANGE, "descriptor %d: N_0 too large", b);
            N = bsk::order_for(q.sigma_r, T);
        }
        Item it;
        bsk::Plan pl;
        if (bsk::make_plan(N, q.sigma_r, o.weight_eps, &pl) != 0)
            return fail(BSK_ERANGE, "descriptor %d: order %d has too many folded orders", b, N);
        if (pl.K == 0) return fail(BSK_EINVAL, "descriptor %d: weight_eps drops every order", b);
        std::memset(&it.im, 0, sizeof(it.im));
        it.im.img = q.img;
        it.im.out = q.out;
        it.im.H = q.H;
        it.im.W = q.W;
        it.im.rh = std::min(q.radius, q.W - 1);
        it.im.rv = std::min(q.radius, q.H - 1);
        it.im.K = pl.K;
        it.im.omega_base = pl.omega_base;
        it.im.delta = pl.delta;
        it.im.start_mode = pl.start_mode;
        it.v.assign(pl.v, pl.v + pl.K);
        max_rh = std::max(max_rh, it.im.rh);
        items.push_back(std::move(it));
    }
    int block = o.block;
    if (block == 0) block = (max_rh <= 64) ? 256 : (max_rh <= 128 ? 512 : 1024);
    if (block != 256 && block != 512 && block != 1024) return fail(BSK_EINVAL, "block must be 256, 512 or 1024");
    if (max_rh > bsk::max_radius_batched(block))
        return fail(BSK_EUNSUPPORTED, "clamped radius %d too large for a %d-lane strip", max_rh, block);
    const int kfull = bsk::chunk_batched_f32(block);
    const int rows = o.strip_h > 0 ? o.strip_h : kBatchRows;
    for (auto &it : items) {
        const int Wt = block - 2 * it.im.rh;
        it.im.strips = (it.im.W + Wt - 1) / Wt;
        it.im.S = std::min(rows, it.im.H);
        // per image: the full pass or its half, whichever pads fewer orders for the cost
        it.im.kc = pick_chunk(it.im.K, kfull);
        const int kc = it.im.kc;
        const int segs = (it.im.H + it.im.S - 1) / it.im.S;
        // work of one unit ~ lanes x (rows + window) x (padded orders + per-pass cost)
        const int passes = (it.im.K + kc - 1) / kc;
        it.cost = (double)it.im.strips * segs * block * (it.im.S + 0.25 * 2 * it.im.rv) *
                  (passes * kc + 2.0 * passes);
    }
    // most expensive images first, so the tail of the persistent loop is short units
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
        const double ua = a.cost / ((double)a.im.strips * ((a.im.H + a.im.S - 1) / a.im.S));
        const double ub = b.cost / ((double)b.im.strips * ((b.im.H + b.im.S - 1) / b.im.S));
        return ua > ub;
    });
    bp->imgs.clear();
    bp->vtab.clear();
    bp->vtabf.clear();
    bp->ws_elems = 0;
    long long units = 0;
    for (auto &it : items) {
        it.im.unit0 = (int)units;
        units += (long long)it.im.strips * ((it.im.H + it.im.S - 1) / it.im.S);
        if (units > (1LL << 30)) return fail(BSK_EINVAL, "too many work units");
        it.im.v_off = (int)bp->vtab.size();
        // pad to whole passes with zero weights
        const int kc = it.im.kc;
        it.im.K = (it.im.K + kc - 1) / kc * kc;
        it.v.resize(it.im.K, 0.0);
        bp->vtab.insert(bp->vtab.end(), it.v.begin(), it.v.end());
        for (double w : it.v) bp->vtabf.push_back((float)w);
        if (it.im.K > kc) {
            it.im.ws_off = bp->ws_elems;
            bp->ws_elems += (long long)bsk::acc_count_forward() * it.im.H * it.im.W;
        } else {
            it.im.ws_off = -1;
        }
        bp->imgs.push_back(it.im);
    }
    bp->total_units = (int)units;
    bp->block = block;
    return BSK_OK;
}

// Device copy of a batch plan: [images | weights | counter], plus workspace.
struct DeviceBatch {
    void *tab = nullptr;
    size_t tab_bytes = 0;
    float *ws = nullptr;
    bsk::BatchArgs args;
};

// Table layout: [images | FP64 weights | FP32 weights | counter], 256-byte aligned parts.
size_t table_bytes(const BatchPlan &bp, size_t *off_v, size_t *off_f, size_t *off_c)
{
    size_t a = bp.imgs.size() * sizeof(bsk::BatchImage);
    a = (a + 255) & ~(size_t)255;
    *off_v = a;
    a += bp.vtab.size() * sizeof(double);
    a = (a + 255) & ~(size_t)255;
    *off_f = a;
    a += bp.vtabf.size() * sizeof(float);
    a = (a + 255) & ~(size_t)255;
    *off_c = a;
    return a + 256;
}

void pack_tables(const BatchPlan &bp, std::vector<char> *host, size_t *off_v, size_t *off_f, size_t *off_c)
{
    const size_t n = table_bytes(bp, off_v, off_f, off_c);
    host->assign(n, 0);
    std::memcpy(host->data(), bp.imgs.data(), bp.imgs.size() * sizeof(bsk::BatchImage));
    std::memcpy(host->data() + *off_v, bp.vtab.data(), bp.vtab.size() * sizeof(double));
    std::memcpy(host->data() + *off_f, bp.vtabf.data(), bp.vtabf.size() * sizeof(float));
}

void set_args(DeviceBatch *db, const BatchPlan &bp, size_t off_v, size_t off_f, size_t off_c)
{
    db->args.imgs = (const bsk::BatchImage *)db->tab;
    db->args.vtab = (const double *)((char *)db->tab + off_v);
    db->args.vtabf = (const float *)((char *)db->tab + off_f);
    db->args.counter = (unsigned *)((char *)db->tab + off_c);
    db->args.ws = db->ws;
    db->args.nimg = (int)bp.imgs.size();
    db->args.total_units = bp.total_units;
}

// Pinned staging for the per-call table upload: one per stream; reused only
// after the copy that last read it has completed.
struct Staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};
std::mutex g_stage_mu;
std::map<std::pair<int, void *>, Staging> g_stage;

int stage_upload(void *stream, const std::vector<char> &tab, void *dev_dst)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging &s = g_stage[{dev, stream}];
    if (s.done) {
        e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    } else {
        e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    if (s.bytes < tab.size()) {
        if (s.host) hipHostFree(s.host);
        s.host = nullptr;
        s.bytes = 0;
        e = hipHostMalloc(&s.host, tab.size(), hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(BSK_ENOMEM, "pinned staging allocation failed");
        }
        s.bytes = tab.size();
    }
    std::memcpy(s.host, tab.data(), tab.size());
    e = hipMemcpyAsync(dev_dst, s.host, tab.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipEventRecord(s.done, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return BSK_OK;
}

int grid_for(int block)
{
    return bsk::wg_per_cu_batched(block) * device_cus();   // every resident workgroup slot
}

// ---------------------------------------------------------------- graphs --
struct GraphEntry {
    std::vector<bsk_image_desc> descs;
    float T;
    bsk_options opt;
    void *stream;
    int dev;
    void *tab = nullptr;
    float *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::map<int, GraphEntry> g_graphs;

bool same_descs(const GraphEntry &g, const bsk_image_desc *d, int B, float T, const bsk_options &o, void *stream,
                int dev)
{
    if ((int)g.descs.size() != B || g.T != T || g.stream != stream || g.dev != dev) return false;
    if (std::memcmp(&g.opt, &o, sizeof(o)) != 0) return false;
    for (int b = 0; b < B; ++b) {
        const bsk_image_desc &x = g.descs[b], &y = d[b];
        if (x.img != y.img || x.out != y.out || x.H != y.H || x.W != y.W || x.radius != y.radius ||
            x.sigma_r != y.sigma_r || x.N != y.N)
            return false;
    }
    return true;
}

void free_graph(GraphEntry &g)
{
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.graph) hipGraphDestroy(g.graph);
    if (g.tab) hipFree(g.tab);
    if (g.ws) hipFree(g.ws);
    g.exec = nullptr;
    g.graph = nullptr;
    g.tab = nullptr;
    g.ws = nullptr;
}

// ------------------------------------------------------------- autotuner --
struct TuneKey {
    int rh, K, H, W, prec;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(rh, K, H, W, prec) < std::tie(o.rh, o.K, o.H, o.W, o.prec);
    }
};
struct TuneVal {
    int block, S, kc;
    double ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
bool g_tune_loaded = false;

void load_tune_file(const char *path)
{
    FILE *f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        TuneKey k;
        TuneVal v;
        if (std::sscanf(line, "{\"rh\": %d, \"K\": %d, \"H\": %d, \"W\": %d, \"prec\": %d, \"block\": %d, \"S\": %d, "
                              "\"kc\": %d, \"ms\": %lf}",
                        &k.rh, &k.K, &k.H, &k.W, &k.prec, &v.block, &v.S, &v.kc, &v.ms) == 9)
            g_tune[k] = v;
    }
    std::fclose(f);
}

void save_tune_file(const char *path)
{
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_tune)
        std::fprintf(f,
                     "{\"rh\": %d, \"K\": %d, \"H\": %d, \"W\": %d, \"prec\": %d, \"block\": %d, \"S\": %d, "
                     "\"kc\": %d, \"ms\": %.6f}\n",
                     kv.first.rh, kv.first.K, kv.first.H, kv.first.W, kv.first.prec, kv.second.block,
                     kv.second.S, kv.second.kc, kv.second.ms);
    std::fclose(f);
}

}  // namespace

namespace bsk {
namespace host {

bool tuned_shape(int rh, int K, int H, int W, int prec, int *block, int *S, int *kc)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        load_tune_file(std::getenv("BSK_TUNE_CACHE"));
    }
    auto it = g_tune.find(TuneKey{rh, K, H, W, prec});
    if (it == g_tune.end()) return false;
    *block = it->second.block;
    *S = it->second.S;
    *kc = it->second.kc;
    return true;
}

}  // namespace host
}  // namespace bsk

extern "C" {

int bilateral_shiftable_batched(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, void *stream)
{
    BatchPlan bp;
    int st = build_batch(descs, B, T, opt, &bp);
    if (st) return st;
    size_t off_v, off_f, off_c;
    std::vector<char> host;
    pack_tables(bp, &host, &off_v, &off_f, &off_c);
    DeviceBatch db;
    if (bp.ws_elems > 0) {
        void *w = nullptr;
        st = get_ws(stream, kWsBatchAcc, (size_t)bp.ws_elems * sizeof(float), &w);
        if (st) return st;
        db.ws = (float *)w;
    }
    st = get_ws(stream, kWsBatchTab, host.size(), &db.tab);
    if (st) return st;
    set_args(&db, bp, off_v, off_f, off_c);
    st = stage_upload(stream, host, db.tab);
    if (st) return st;
    hipError_t e = bsk::launch_batched_f32(db.args, bp.block, grid_for(bp.block), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return BSK_OK;
}

int bilateral_shiftable_batched_graph(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, int key,
                                      void *stream)
{
    if (!stream) return fail(BSK_EINVAL, "graph capture needs a non-default stream");
    bsk_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
        if (!descs || B < 1 || !same_descs(it->second, descs, B, T, o, stream, dev))
            return fail(BSK_EINVAL, "graph key %d was captured for different descriptors", key);
        e = hipGraphLaunch(it->second.exec, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return BSK_OK;
    }
    BatchPlan bp;
    int st = build_batch(descs, B, T, opt, &bp);
    if (st) return st;
    size_t off_v, off_f, off_c;
    std::vector<char> host;
    pack_tables(bp, &host, &off_v, &off_f, &off_c);
    GraphEntry g;
    g.descs.assign(descs, descs + B);
    g.T = T;
    g.opt = o;
    g.stream = stream;
    g.dev = dev;
    // the graph owns its tables and workspace, uploaded once before capture
    e = hipMalloc(&g.tab, host.size());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BSK_ENOMEM, "graph table allocation failed");
    }
    if (bp.ws_elems > 0) {
        e = hipMalloc((void **)&g.ws, (size_t)bp.ws_elems * sizeof(float));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_graph(g);
            return fail(BSK_ENOMEM, "graph workspace allocation failed");
        }
    }
    e = hipMemcpy(g.tab, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(e, "hipMemcpy");
    }
    DeviceBatch db;
    db.tab = g.tab;
    db.ws = g.ws;
    set_args(&db, bp, off_v, off_f, off_c);
    e = hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    hipError_t le = bsk::launch_batched_f32(db.args, bp.block, grid_for(bp.block), (hipStream_t)stream);
    e = hipStreamEndCapture((hipStream_t)stream, &g.graph);
    if (le != hipSuccess || e != hipSuccess) {
        free_graph(g);
        return hip_fail(le != hipSuccess ? le : e, "graph capture");
    }
    e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    e = hipGraphLaunch(g.exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(e, "hipGraphLaunch");
    }
    g_graphs[key] = std::move(g);
    return BSK_OK;
}

// Release hook for the batched state, called by bsk_release().
void bsk_release_batched(void)
{
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto &kv : g_graphs) free_graph(kv.second);
        g_graphs.clear();
    }
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (auto &kv : g_stage) {
        if (kv.second.done) {
            hipEventSynchronize(kv.second.done);
            hipEventDestroy(kv.second.done);
        }
        if (kv.second.host) hipHostFree(kv.second.host);
    }
    g_stage.clear();
}

int bsk_autotune(const void *img, int H, int W, int radius, float sigma_r, float T, void *out,
                 const bsk_options *opt, const char *path, void *stream, int *best_block, int *best_rows,
                 int *best_chunk, double *best_ms)
{
    if (!img || !out) return fail(BSK_EINVAL, "null pointer");
    bsk_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    o.block = 0;
    o.strip_h = 0;
    o.order_chunk = 0;
    if (o.spatial_N != 0) return fail(BSK_EUNSUPPORTED, "the autotuner covers the box spatial kernel");
    if (o.range_kernel != BSK_RANGE_COS) return fail(BSK_EUNSUPPORTED, "the autotuner covers the raised cosine");
    Resolved base;
    int st = resolve(H, W, radius, sigma_r, T, &o, &base);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune_loaded) {
            g_tune_loaded = true;
            load_tune_file(std::getenv("BSK_TUNE_CACHE"));
        }
        load_tune_file(path);
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(BSK_EHIP, "hipEventCreate failed");
    const int blocks[3] = {256, 512, 1024};
    const int rows[9] = {16, 24, 32, 48, 64, 96, 128, 192, 256};
    TuneVal best{0, 0, 0, 1e30};
    for (int b : blocks) {
        if (b - 2 * base.rh < b / 4 && !(b == 1024 && base.rh <= 511)) continue;
        if (b - 2 * base.rh < 1) continue;
        const int full = bsk::chunk_forward_f32(b);
        const int kcs[2] = {full, full / 2};
        for (int kc : kcs) {
            // the FP64 forward has a single pass size
            if (base.prec == BSK_FP64 && kc != full) continue;
            for (int S : rows) {
                if (S > H && S != rows[0]) continue;
                bsk_options c = o;
                c.block = b;
                c.strip_h = S;
                c.order_chunk = base.prec == BSK_FP64 ? 0 : kc;
                float ms_min = 1e30f;
                for (int rep = 0; rep < 4; ++rep) {
                    if (hipEventRecord(e0, (hipStream_t)stream) != hipSuccess) break;
                    st = bilateral_shiftable_ex(img, H, W, radius, sigma_r, T, out, &c, stream);
                    if (st) break;
                    if (hipEventRecord(e1, (hipStream_t)stream) != hipSuccess) break;
                    if (hipEventSynchronize(e1) != hipSuccess) break;
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, e0, e1);
                    if (rep > 0 && ms < ms_min) ms_min = ms;   // first run is a warm-up
                }
                if (st) {
                    hipEventDestroy(e0);
                    hipEventDestroy(e1);
                    return st;
                }
                if (ms_min < best.ms) best = TuneVal{b, S, c.order_chunk, (double)ms_min};
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best.block == 0) return fail(BSK_EUNSUPPORTED, "no launch shape fits this request");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[TuneKey{base.rh, base.plan.K, H, W, base.prec}] = best;
        save_tune_file(path);
    }
    if (best_block) *best_block = best.block;
    if (best_rows) *best_rows = best.S;
    if (best_chunk) *best_chunk = best.kc;
    if (best_ms) *best_ms = best.ms;
    return BSK_OK;
}

}  // extern "C"
