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
    std::vector<int> rows, chunk;   // per descriptor, in descriptor order: rows per unit, orders per pass
    std::vector<int> rbucket, kbucket;
    int qstart[bsk::kBatchQueues + 1] = {};   // per-XCD queues of units (BatchArgs::qstart)
};

constexpr int kBatchRows = 96;   // default output rows per work unit (64: 1% slower on the 256-image batch)

// Tuning buckets of the batched launch: clamped radius 0, 1, 2-3, 4-7, 8-15,
// ... (bit length) and folded orders 1, 2, 3-4, 5-8, 9-16, ... (ceil log2).
int radius_bucket(int rh)
{
    int b = 0;
    while (b < 30 && (1 << b) <= rh) ++b;
    return b;
}
int order_bucket(int K)
{
    int b = 0;
    while (b < 30 && (1 << b) < K) ++b;
    return b;
}

// Batched launch shapes measured by bsk_autotune_batched: per (radius bucket,
// order bucket, precision, lanes) the rows per work unit and orders per pass,
// and per (largest radius bucket of a batch, precision) the lanes per workgroup.
struct BatchTuneKey {
    int rb, kb, prec, block;
    bool operator<(const BatchTuneKey &o) const
    {
        return std::tie(rb, kb, prec, block) < std::tie(o.rb, o.kb, o.prec, o.block);
    }
};
struct BatchTuneVal {
    int S, kc;
    double ms;
};
struct BatchBlockKey {
    int rb, prec;
    bool operator<(const BatchBlockKey &o) const { return std::tie(rb, prec) < std::tie(o.rb, o.prec); }
};
struct BatchBlockVal {
    int block;
    double ms;
};
// What the tuner's sweep imposes on build_batch: lanes (0: the usual choice),
// per (radius bucket, order bucket) rows and orders per pass, and whether the
// measured table is consulted at all.
struct BatchShapeOverride {
    bool use_table = true;
    int block = 0;
    std::map<std::pair<int, int>, std::pair<int, int>> shape;
};
bool batch_tuned_block(int rb, int prec, int *block);
bool batch_tuned_shape(int rb, int kb, int prec, int block, int *S, int *kc);

int build_batch(const bsk_image_desc *d, int B, float T, const bsk_options *opt, BatchPlan *bp,
                const BatchShapeOverride *ovr = nullptr)
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

    if (o.order_chunk < 0) return fail(BSK_EINVAL, "bad options");
    struct Item {
        bsk::BatchImage im;
        std::vector<double> v;
        double cost;
        int idx, rb, kb;
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
        it.idx = b;
        it.rb = radius_bucket(std::max(it.im.rh, it.im.rv));
        it.kb = order_bucket(pl.K);
        max_rh = std::max(max_rh, it.im.rh);
        items.push_back(std::move(it));
    }
    const bool table = !ovr || ovr->use_table;
    constexpr int prec = BSK_FP32;
    int block = o.block;
    if (block == 0 && ovr && ovr->block) block = ovr->block;
    if (block == 0 && table) {
        int rbmax = 0;
        for (const auto &it : items) rbmax = std::max(rbmax, it.rb);
        int tb = 0;
        if (batch_tuned_block(rbmax, prec, &tb) && max_rh <= bsk::max_radius_batched(tb)) block = tb;
    }
    if (block == 0) block = (max_rh <= 64) ? 256 : (max_rh <= 128 ? 512 : 1024);
    if (block != 256 && block != 512 && block != 1024) return fail(BSK_EINVAL, "block must be 256, 512 or 1024");
    if (max_rh > bsk::max_radius_batched(block))
        return fail(BSK_EUNSUPPORTED, "clamped radius %d too large for a %d-lane strip", max_rh, block);
    const int kfull = bsk::chunk_batched_f32(block);
    const int kmid = bsk::mid_chunk_batched_f32(block);
    auto pass_size = [&](int kc) { return kc == kfull || kc == kfull / 2 || (kmid > 0 && kc == kmid); };
    if (o.order_chunk != 0 && !pass_size(o.order_chunk)) {
        if (kmid > 0)
            return fail(BSK_EINVAL, "order_chunk %d is not a pass size (%d, %d or %d) of the %d-lane batched kernel",
                        o.order_chunk, kfull, kmid, kfull / 2, block);
        return fail(BSK_EINVAL, "order_chunk %d is not a pass size (%d or %d) of the %d-lane batched kernel",
                    o.order_chunk, kfull, kfull / 2, block);
    }
    bp->rows.assign(B, 0);
    bp->chunk.assign(B, 0);
    bp->rbucket.assign(B, 0);
    bp->kbucket.assign(B, 0);
    for (auto &it : items) {
        const int Wt = block - 2 * it.im.rh;
        it.im.strips = (it.im.W + Wt - 1) / Wt;
        // rows per unit and orders per pass: the options, else the tuner's sweep,
        // else the measured table, else the defaults (the full pass or its half,
        // whichever pads fewer orders for the cost)
        int rows = kBatchRows, kc = pick_chunk(it.im.K, kfull, 0, kmid);
        int ts = 0, tk = 0;
        if (ovr) {
            auto f = ovr->shape.find({it.rb, it.kb});
            if (f != ovr->shape.end()) {
                ts = f->second.first;
                tk = f->second.second;
            }
        }
        if (!ts && table) batch_tuned_shape(it.rb, it.kb, prec, block, &ts, &tk);
        if (ts > 0) rows = ts;
        if (tk > 0 && pass_size(tk)) kc = tk;
        if (o.strip_h > 0) rows = o.strip_h;
        if (o.order_chunk > 0) kc = o.order_chunk;
        it.im.S = std::min(rows, it.im.H);
        it.im.kc = kc;
        bp->rows[it.idx] = it.im.S;
        bp->chunk[it.idx] = kc;
        bp->rbucket[it.idx] = it.rb;
        bp->kbucket[it.idx] = it.kb;
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
    // One queue per XCD: images go, most expensive unit first, to the queue with
    // the least work so far (so every queue also ends with its cheapest units),
    // and each queue's images are numbered contiguously.
    {
        double load[bsk::kBatchQueues] = {};
        std::vector<int> queue(items.size());
        for (size_t i = 0; i < items.size(); ++i) {
            int best = 0;
            for (int q = 1; q < bsk::kBatchQueues; ++q)
                if (load[q] < load[best]) best = q;
            queue[i] = best;
            load[best] += items[i].cost;
        }
        std::vector<Item> byq;
        byq.reserve(items.size());
        for (int q = 0; q < bsk::kBatchQueues; ++q)
            for (size_t i = 0; i < items.size(); ++i)
                if (queue[i] == q) byq.push_back(std::move(items[i]));
        // queue boundaries in image indices, turned into unit indices below
        int qi = 0;
        bp->qstart[0] = 0;
        for (int q = 0; q < bsk::kBatchQueues; ++q) {
            for (size_t i = 0; i < queue.size(); ++i) qi += queue[i] == q;
            bp->qstart[q + 1] = qi;   // image index where queue q + 1 begins
        }
        items = std::move(byq);
    }
    long long units = 0;
    std::vector<int> img_unit0;
    img_unit0.reserve(items.size() + 1);
    for (auto &it : items) {
        it.im.unit0 = (int)units;
        img_unit0.push_back((int)units);
        const long long nu = (long long)it.im.strips * ((it.im.H + it.im.S - 1) / it.im.S);
        units += nu;
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
    img_unit0.push_back((int)units);
    for (int q = 0; q <= bsk::kBatchQueues; ++q) bp->qstart[q] = img_unit0[bp->qstart[q]];
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
    for (int q = 0; q <= bsk::kBatchQueues; ++q) db->args.qstart[q] = bp.qstart[q];
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
        if (s.host) (void)hipHostFree(s.host);
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
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.tab) (void)hipFree(g.tab);
    if (g.ws) (void)hipFree(g.ws);
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
std::mutex g_tune_mu;   // guards every table below
std::map<TuneKey, TuneVal> g_tune;
std::map<BatchTuneKey, BatchTuneVal> g_btune;
std::map<BatchBlockKey, BatchBlockVal> g_bblock;
bool g_tune_loaded = false;

// Cache file: JSON lines of three kinds (single-image shapes, batched shapes
// per bucket, batched lanes per largest radius bucket).  Returns false if the
// file cannot be opened; lines of no known kind are skipped.
bool load_tune_file(const char *path)
{
    FILE *f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return false;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        TuneKey k;
        TuneVal v;
        BatchTuneKey bk;
        BatchTuneVal bv;
        BatchBlockKey lk;
        BatchBlockVal lv;
        if (std::sscanf(line, "{\"rh\": %d, \"K\": %d, \"H\": %d, \"W\": %d, \"prec\": %d, \"block\": %d, \"S\": %d, "
                              "\"kc\": %d, \"ms\": %lf}",
                        &k.rh, &k.K, &k.H, &k.W, &k.prec, &v.block, &v.S, &v.kc, &v.ms) == 9)
            g_tune[k] = v;
        else if (std::sscanf(line, "{\"batched_rb\": %d, \"kb\": %d, \"prec\": %d, \"block\": %d, \"S\": %d, "
                                   "\"kc\": %d, \"ms\": %lf}",
                             &bk.rb, &bk.kb, &bk.prec, &bk.block, &bv.S, &bv.kc, &bv.ms) == 7)
            g_btune[bk] = bv;
        else if (std::sscanf(line, "{\"batched_block_rb\": %d, \"prec\": %d, \"block\": %d, \"ms\": %lf}", &lk.rb,
                             &lk.prec, &lv.block, &lv.ms) == 4)
            g_bblock[lk] = lv;
    }
    std::fclose(f);
    return true;
}

bool save_tune_file(const char *path)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "w");
    if (!f) return false;
    for (auto &kv : g_tune)
        std::fprintf(f,
                     "{\"rh\": %d, \"K\": %d, \"H\": %d, \"W\": %d, \"prec\": %d, \"block\": %d, \"S\": %d, "
                     "\"kc\": %d, \"ms\": %.6f}\n",
                     kv.first.rh, kv.first.K, kv.first.H, kv.first.W, kv.first.prec, kv.second.block,
                     kv.second.S, kv.second.kc, kv.second.ms);
    for (auto &kv : g_btune)
        std::fprintf(f, "{\"batched_rb\": %d, \"kb\": %d, \"prec\": %d, \"block\": %d, \"S\": %d, \"kc\": %d, "
                        "\"ms\": %.6f}\n",
                     kv.first.rb, kv.first.kb, kv.first.prec, kv.first.block, kv.second.S, kv.second.kc,
                     kv.second.ms);
    for (auto &kv : g_bblock)
        std::fprintf(f, "{\"batched_block_rb\": %d, \"prec\": %d, \"block\": %d, \"ms\": %.6f}\n", kv.first.rb,
                     kv.first.prec, kv.second.block, kv.second.ms);
    const bool ok = std::ferror(f) == 0;
    return std::fclose(f) == 0 && ok;
}

// The environment's cache file, read once at first use (caller holds g_tune_mu).
void ensure_tune_loaded()
{
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        load_tune_file(std::getenv("BSK_TUNE_CACHE"));
    }
}

bool batch_tuned_block(int rb, int prec, int *block)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_tune_loaded();
    auto it = g_bblock.find(BatchBlockKey{rb, prec});
    if (it == g_bblock.end()) return false;
    *block = it->second.block;
    return true;
}

bool batch_tuned_shape(int rb, int kb, int prec, int block, int *S, int *kc)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_tune_loaded();
    auto it = g_btune.find(BatchTuneKey{rb, kb, prec, block});
    if (it == g_btune.end()) return false;
    *S = it->second.S;
    *kc = it->second.kc;
    return true;
}

}  // namespace

namespace bsk {
namespace host {

bool tuned_shape(int rh, int K, int H, int W, int prec, int *block, int *S, int *kc)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_tune_loaded();
    auto it = g_tune.find(TuneKey{rh, K, H, W, prec});
    if (it == g_tune.end()) return false;
    *block = it->second.block;
    *S = it->second.S;
    *kc = it->second.kc;
    return true;
}

}  // namespace host
}  // namespace bsk

namespace {
int run_batched(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, void *stream,
                const BatchShapeOverride *ovr);
}

extern "C" {

int bilateral_shiftable_batched(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, void *stream)
{
    return run_batched(descs, B, T, opt, stream, nullptr);
}

}  // extern "C"

namespace {

int run_batched(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, void *stream,
                const BatchShapeOverride *ovr)
{
    BatchPlan bp;
    int st = build_batch(descs, B, T, opt, &bp, ovr);
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

}  // namespace

extern "C" {

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
            (void)hipEventSynchronize(kv.second.done);
            (void)hipEventDestroy(kv.second.done);
        }
        if (kv.second.host) (void)hipHostFree(kv.second.host);
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
        ensure_tune_loaded();
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
        // every pass size of the stack at this lane count (the FP64 forward has
        // a single one, chosen by the library)
        int kcs[bsk::kMaxForwardChunks];
        const int nkc = base.prec == BSK_FP64 ? 1 : bsk::forward_chunks_f32(b, base.prec, base.kahan, base.rh, kcs);
        if (base.prec == BSK_FP64) kcs[0] = 0;
        for (int ik = 0; ik < nkc; ++ik) {
            const int kc = kcs[ik];
            for (int S : rows) {
                if (S > H && S != rows[0]) continue;
                bsk_options c = o;
                c.block = b;
                c.strip_h = S;
                c.order_chunk = kc;
                float ms_min = 1e30f;
                for (int rep = 0; rep < 4; ++rep) {
                    if (hipEventRecord(e0, (hipStream_t)stream) != hipSuccess) break;
                    st = bilateral_shiftable_ex(img, H, W, radius, sigma_r, T, out, &c, stream);
                    if (st) break;
                    if (hipEventRecord(e1, (hipStream_t)stream) != hipSuccess) break;
                    if (hipEventSynchronize(e1) != hipSuccess) break;
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) break;
                    if (rep > 0 && ms < ms_min) ms_min = ms;   // first run is a warm-up
                }
                if (st) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return st;
                }
                if (ms_min < best.ms) best = TuneVal{b, S, c.order_chunk, (double)ms_min};
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
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

int bsk_batched_shape(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, int *block, int *rows,
                      int *chunk)
{
    BatchPlan bp;
    const int st = build_batch(descs, B, T, opt, &bp);
    if (st) return st;
    if (block) *block = bp.block;
    for (int b = 0; b < B; ++b) {
        if (rows) rows[b] = bp.rows[b];
        if (chunk) chunk[b] = bp.chunk[b];
    }
    return BSK_OK;
}

int bsk_autotune_batched(const bsk_image_desc *descs, int B, float T, const bsk_options *opt, const char *path,
                         void *stream, int *best_block, double *best_ms)
{
    bsk_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    o.block = 0;
    o.strip_h = 0;
    o.order_chunk = 0;
    // the plan with the defaults validates the request before anything is timed
    BatchShapeOverride ovr;
    ovr.use_table = false;
    BatchPlan base;
    int st = build_batch(descs, B, T, &o, &base, &ovr);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        ensure_tune_loaded();
        load_tune_file(path);
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(BSK_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(BSK_EHIP, "hipEventCreate failed");
    }
    // one warm-up launch, then the fastest of three
    auto time_it = [&](const BatchShapeOverride &v, double *ms) -> int {
        double best = 1e30;
        for (int rep = 0; rep < 4; ++rep) {
            hipError_t e = hipEventRecord(e0, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
            const int r = run_batched(descs, B, T, &o, stream, &v);
            if (r) return r;
            e = hipEventRecord(e1, (hipStream_t)stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            float t = 0.f;
            e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            if (rep > 0 && t < best) best = t;
        }
        *ms = best;
        return BSK_OK;
    };
    int max_rh = 0, rbmax = 0;
    // buckets present, with their pixel counts (most pixels first)
    std::map<std::pair<int, int>, double> pix;
    std::map<std::pair<int, int>, int> hmax;
    for (int b = 0; b < B; ++b) {
        const int rh = std::min(descs[b].radius, descs[b].W - 1);
        max_rh = std::max(max_rh, rh);
        rbmax = std::max(rbmax, base.rbucket[b]);
        const auto key = std::make_pair(base.rbucket[b], base.kbucket[b]);
        pix[key] += (double)descs[b].H * descs[b].W;
        hmax[key] = std::max(hmax[key], descs[b].H);
    }
    std::vector<std::pair<double, std::pair<int, int>>> order;
    for (auto &kv : pix) order.push_back({kv.second, kv.first});
    std::sort(order.begin(), order.end(), [](const auto &a, const auto &b) { return a.first > b.first; });

    // lanes per workgroup first (with the default rows and passes), then a
    // coordinate sweep over the buckets' rows and pass sizes at those lanes
    double best = 1e30;
    int bblock = 0;
    for (int blk : {256, 512, 1024}) {
        if (max_rh > bsk::max_radius_batched(blk)) continue;
        BatchShapeOverride v = ovr;
        v.block = blk;
        double ms = 0.0;
        st = time_it(v, &ms);
        if (st) break;
        if (ms < best) {
            best = ms;
            bblock = blk;
        }
    }
    ovr.block = bblock;
    const int kfull = bblock ? bsk::chunk_batched_f32(bblock) : 0;
    const int rows_c[7] = {32, 48, 64, 96, 128, 192, 256};
    for (size_t q = 0; !st && q < order.size(); ++q) {
        const auto key = order[q].second;
        std::pair<int, int> keep{0, 0};
        for (int si = 0; si < 7; ++si) {
            const int S = rows_c[si];
            // units taller than the bucket's tallest image are all the same shape
            if (si > 0 && rows_c[si - 1] >= hmax[key]) break;
            const int kmid = bblock ? bsk::mid_chunk_batched_f32(bblock) : 0;
            for (int kc : {kfull, kmid, kfull / 2}) {
                if (kc <= 0) continue;
                BatchShapeOverride v = ovr;
                v.shape[key] = {S, kc};
                double ms = 0.0;
                st = time_it(v, &ms);
                if (st) break;
                if (ms < best) {
                    best = ms;
                    keep = {S, kc};
                }
            }
            if (st) break;
        }
        if (keep.first) ovr.shape[key] = keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    // the lanes and the buckets' shapes the sweep settled on (buckets it left
    // at the defaults record nothing), stored for later calls and written to `path`
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_bblock[BatchBlockKey{rbmax, BSK_FP32}] = BatchBlockVal{bblock, best};
        for (auto &kv : ovr.shape)
            g_btune[BatchTuneKey{kv.first.first, kv.first.second, BSK_FP32, bblock}] =
                BatchTuneVal{kv.second.first, kv.second.second, best};
        if (path && !save_tune_file(path)) return fail(BSK_EINVAL, "cannot write the tune cache %s", path);
    }
    if (best_block) *best_block = bblock;
    if (best_ms) *best_ms = best;
    return BSK_OK;
}

int bsk_tune_cache_load(const char *path)
{
    if (!path) return fail(BSK_EINVAL, "null path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_tune_loaded();
    if (!load_tune_file(path)) return fail(BSK_EINVAL, "cannot read the tune cache %s", path);
    return BSK_OK;
}

int bsk_tune_cache_save(const char *path)
{
    if (!path) return fail(BSK_EINVAL, "null path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_tune_loaded();
    if (!save_tune_file(path)) return fail(BSK_EINVAL, "cannot write the tune cache %s", path);
    return BSK_OK;
}

int bsk_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_loaded = true;   // the environment's file is not re-read after a clear
    g_tune.clear();
    g_btune.clear();
    g_bblock.clear();
    return BSK_OK;
}

}  // extern "C"
