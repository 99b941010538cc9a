// Batch entry points: many independent Vegas integrations run together (see
// include/vegas.h).  All iterations of all problems are recorded once as a
// HIP graph and replayed with one graph launch.  The tile size (events per
// work item, which also fixes events per thread) is chosen at plan time by
// timing candidate schedules on the batch itself.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "capi_util.hpp"
#include "vegas_internal.hpp"

using namespace vegas;

namespace {

constexpr int kBatchMaxIter = 1024;
constexpr int kMaxProblems = 65535;
const uint64_t kTileCandidates[] = {1u << 13, 1u << 14, 1u << 15, 1u << 16, 1u << 17};
constexpr uint64_t kTileMin = 1u << 13;
constexpr int kTuneWarmRuns = 3;  // untimed schedule timings before the tuning's own

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

int dmax_of(int d)
{
    if (d <= 4) return 4;
    if (d <= 8) return 8;
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    return 64;
}

// Byte layout of a batch workspace.
struct BatchLayout {
    size_t probs, items, queue, params, cst, records, rec_flag, results;
    std::vector<size_t> edges, tab64, tab32, thr, last;  // per problem
    size_t partials;
    size_t total;
    size_t max_items;
    size_t partial_doubles;
};

BatchLayout batch_layout(const vegas_desc* descs, const int64_t* n_events, int n)
{
    BatchLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = a256(o + bytes); return at; };
    size_t max_items = 0, pd = 0;
    for (int p = 0; p < n; ++p) {
        const size_t it = (size_t(n_events[p]) + kTileMin - 1) / kTileMin;
        max_items += it;
        pd += it * size_t(2 + descs[p].dim * descs[p].n_bins);
    }
    L.max_items = max_items;
    L.partial_doubles = pd;
    L.probs = take(sizeof(BatchProblem) * n);
    L.items = take(sizeof(BatchItem) * max_items);
    L.queue = take(256);
    L.params = take(sizeof(double) * kMaxParams * n);
    L.cst = take(sizeof(DevConst) * n);
    L.records = take(sizeof(double) * 2 * kBatchMaxIter * n);
    L.rec_flag = take(sizeof(int32_t) * kBatchMaxIter * n);
    L.results = take(sizeof(DevResult) * n);
    for (int p = 0; p < n; ++p) {
        const int d = descs[p].dim, N = descs[p].n_bins;
        L.edges.push_back(take(sizeof(double) * d * (N + 1)));
        L.tab64.push_back(take(sizeof(double) * 2 * d * N));
        L.tab32.push_back(take(sizeof(float) * 4 * d * N));
        L.thr.push_back(take(sizeof(uint64_t) * d));
        L.last.push_back(take(sizeof(double) * (2 + d * N)));
    }
    L.partials = take(sizeof(double) * pd);
    L.total = o;
    return L;
}

vegas_status check_batch(const vegas_desc* descs, const int64_t* n_events, int32_t n)
{
    if (!descs || !n_events) return fail(VEGAS_EINVAL, "descs / n_events is NULL");
    if (n < 1 || n > kMaxProblems) return fail(VEGAS_EINVAL, "batch size must be in [1, %d]", kMaxProblems);
    for (int p = 0; p < n; ++p) {
        vegas_status st = check_desc(&descs[p]);
        if (st != VEGAS_OK) return fail(st, "problem %d: %s", p, g_err.c_str());
        if (descs[p].integrand == VEGAS_USER)
            return fail(VEGAS_EUNSUPPORTED, "problem %d: user integrands run as single contexts, not in batches", p);
        if (descs[p].integrand != descs[0].integrand || descs[p].precision != descs[0].precision)
            return fail(VEGAS_EINVAL, "problem %d: all problems of a batch share one integrand kind and precision", p);
        if (n_events[p] < 2 || n_events[p] > (int64_t(1) << 40))
            return fail(VEGAS_EINVAL, "problem %d: n_events must be in [2, 2^40]", p);
    }
    return VEGAS_OK;
}

}  // namespace

struct vegas_batch {
    int n = 0, kind = 0, prec = 0, dmax = 0, n_iter = 0, n_adapt = 0;
    void* ws = nullptr;
    BatchLayout L;
    std::vector<BatchProblem> probs;
    std::vector<int> dims, bins;
    std::vector<int64_t> events;
    // one launch of the event kernel per dimension bucket present
    struct Bucket {
        int dmax = 0;
        int lo = 0, hi = 0;  // item range (set with the schedule)
        size_t lds = 0;
        int blocks = 0;
        int threads = kBlock;
        int hrep_log2 = 0;
        int fix_l2 = 0;         // the histogram launch's fixed layout (log2 of its replicas), 0: general
        double tuned_ms = 0.0;  // its launches' time in one run (n_adapt with, the rest without histograms)
    };
    std::vector<Bucket> buckets;
    bool tuned_from_cache = false;
    int blocks = 0;  // the largest bucket launch (reported by vegas_batch_schedule)
    uint64_t tile = 0;
    int n_items = 0;
    double tuned_ms = 0.0;
    hipStream_t priv = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    int next_step = 0;  // the iteration vegas_batch_step runs next (0 after a graph run)
    size_t max_pstride = 0;

    char* at(size_t off) const { return static_cast<char*>(ws) + off; }
    BatchArgs args() const
    {
        BatchArgs a{};
        a.probs = reinterpret_cast<const BatchProblem*>(at(L.probs));
        a.items = reinterpret_cast<const BatchItem*>(at(L.items));
        a.partials = reinterpret_cast<double*>(at(L.partials));
        a.queue = reinterpret_cast<uint32_t*>(at(L.queue));
        a.item_lo = 0;
        a.item_hi = n_items;
        a.n_probs = n;
        a.hrep_log2 = 0;
        return a;
    }
};

namespace {

// Work items for tile size T, in decreasing cost (dimension), then problem,
// then event order; each problem's items are contiguous, and so are its rows.
void build_items(vegas_batch* b, uint64_t T, std::vector<BatchItem>& items)
{
    std::vector<int> order(b->n);
    for (int p = 0; p < b->n; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->dims[x] > b->dims[y]; });
    items.clear();
    uint64_t row = 0;
    for (int p : order) {
        BatchProblem& pr = b->probs[p];
        pr.first_item = int(items.size());
        pr.row0 = row;
        const uint64_t M = uint64_t(b->events[p]);
        for (uint64_t e0 = 0; e0 < M; e0 += T) {
            BatchItem it{};
            it.prob = p;
            it.e0 = e0;
            it.n = std::min<uint64_t>(T, M - e0);
            it.row_off = row;
            row += uint64_t(pr.pstride);
            items.push_back(it);
        }
        pr.n_items = int(items.size()) - pr.first_item;
    }
    b->n_items = int(items.size());
    // dimensions run in decreasing order, so each bucket's items are contiguous
    for (auto& bk : b->buckets) {
        bk.lo = int(items.size());
        bk.hi = 0;
    }
    for (int k = 0; k < int(items.size()); ++k) {
        const int dm = dmax_of(b->dims[items[k].prob]);
        for (auto& bk : b->buckets)
            if (bk.dmax == dm) {
                bk.lo = std::min(bk.lo, k);
                bk.hi = std::max(bk.hi, k + 1);
            }
    }
}

vegas_status upload_schedule(vegas_batch* b, uint64_t T)
{
    std::vector<BatchItem> items;
    build_items(b, T, items);
    if (items.size() > b->L.max_items) return fail(VEGAS_EINVAL, "internal: too many items");
    VEGAS_HIP(hipMemcpyAsync(b->at(b->L.items), items.data(), sizeof(BatchItem) * items.size(),
                             hipMemcpyHostToDevice, b->priv));
    VEGAS_HIP(hipMemcpyAsync(b->at(b->L.probs), b->probs.data(), sizeof(BatchProblem) * b->n,
                             hipMemcpyHostToDevice, b->priv));
    VEGAS_HIP(hipStreamSynchronize(b->priv));  // the host vectors go out of scope
    b->tile = T;
    return VEGAS_OK;
}

// One iteration of every problem: persistent event kernel, then the per-problem
// reduction (records iteration k; refines while k < n_adapt).
// ev (tuning only): HIP events recorded before and after each bucket's launch.
vegas_status enqueue_iteration(vegas_batch* b, int k, hipStream_t s, const hipEvent_t* ev = nullptr)
{
    BatchArgs a = b->args();
    a.t = uint32_t(k);
    // accumulation iterations run on a frozen grid: no histograms
    const bool adapt = k < b->n_adapt;
    for (size_t q = 0; q < b->buckets.size(); ++q) {
        const auto& bk = b->buckets[q];
        BatchArgs ab = a;
        ab.queue = a.queue + q;
        ab.item_lo = bk.lo;
        ab.item_hi = bk.hi;
        ab.hrep_log2 = bk.hrep_log2;
        if (ev) VEGAS_HIP(hipEventRecord(ev[2 * q], s));
        VEGAS_HIP(launch_batch_sample(b->prec, b->kind, bk.dmax, bk.lds, ab, bk.blocks, bk.threads, adapt, bk.fix_l2, s));
        if (ev) VEGAS_HIP(hipEventRecord(ev[2 * q + 1], s));
    }
    const int flags = adapt ? (MERGE_REFINE | MERGE_NO_COMBINE) : MERGE_NO_HIST;
    VEGAS_HIP(launch_batch_finish(a, b->dmax, b->kind, k, flags, s));
    return VEGAS_OK;
}

// A launch shape of a bucket's event kernel.
struct Shape {
    int threads, l2;  // threads per block, log2 of the histogram replicas
    size_t lds;       // dynamic LDS per block
    int blocks, bpc;  // blocks of the launch (resident ones on every CU), blocks per CU
    int fix_l2;       // the fixed histogram layout (= l2), or 0
};

void apply_shape(vegas_batch::Bucket& bk, const Shape& sh)
{
    bk.threads = sh.threads;
    bk.hrep_log2 = sh.l2;
    bk.lds = sh.lds;
    bk.blocks = sh.blocks;
    bk.fix_l2 = sh.fix_l2;
}

int env_int(const char* name)
{
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : 0;
}

struct Timer {
    std::vector<hipEvent_t> ev;
    hipError_t init(int n)
    {
        ev.assign(size_t(n), nullptr);
        for (auto& e : ev) {
            const hipError_t he = hipEventCreate(&e);
            if (he != hipSuccess) {
                e = nullptr;
                return he;
            }
        }
        return hipSuccess;
    }
    ~Timer()
    {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Time of each bucket's launches in one run under the current schedule:
// n_adapt times its launch with histograms plus (n_iter - n_adapt) times its
// launch without, each the fastest of two launches after a warm-up
// iteration.  The iterations timed here leave the problems' state
// (grids, records) arbitrary: the recorded run restarts every problem.
vegas_status time_schedule(vegas_batch* b, Timer& tm, std::vector<double>& per)
{
    hipStream_t s = b->priv;
    const size_t nb = b->buckets.size();
    per.assign(nb, 0.0);
    VEGAS_HIP(launch_batch_reset(b->args(), b->dmax, kBatchMaxIter, b->kind, s));
    vegas_status st = enqueue_iteration(b, 0, s);
    if (st != VEGAS_OK) return st;
    const int kinds[2] = {b->n_adapt > 0 ? 0 : -1, b->n_adapt < b->n_iter ? b->n_adapt : -1};
    const double weight[2] = {double(b->n_adapt), double(b->n_iter - b->n_adapt)};
    for (int w = 0; w < 2; ++w) {
        if (kinds[w] < 0) continue;
        std::vector<double> best(nb, 1e300);
        for (int r = 0; r < 2; ++r) {
            if ((st = enqueue_iteration(b, kinds[w], s, tm.ev.data())) != VEGAS_OK) return st;
            VEGAS_HIP(hipEventSynchronize(tm.ev[2 * nb - 1]));
            for (size_t q = 0; q < nb; ++q) {
                float ms = 0.f;
                VEGAS_HIP(hipEventElapsedTime(&ms, tm.ev[2 * q], tm.ev[2 * q + 1]));
                best[q] = std::min(best[q], double(ms));
            }
        }
        for (size_t q = 0; q < nb; ++q) per[q] += weight[w] * best[q];
    }
    VEGAS_HIP(hipStreamSynchronize(s));
    return VEGAS_OK;
}

// Tuning-cache key: the device (architecture, compute units) and the batch
// (precision, integrand, sizes of every problem, iteration counts).
std::string tune_key(const vegas_batch* b, int dev, int cus)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    uint64_t h = 1469598103934665603ull;  // FNV-1a over (d, N, M) of every problem
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    for (int p = 0; p < b->n; ++p) {
        mix(uint64_t(b->dims[p]));
        mix(uint64_t(b->bins[p]));
        mix(uint64_t(b->events[p]));
    }
    std::ostringstream o;
    o << "vegas-batch-v1 " << arch << " cu" << cus << " p" << b->prec << " k" << b->kind << " n" << b->n << " i"
      << b->n_iter << " a" << b->n_adapt << " h" << std::hex << h;
    return o.str();
}

// A cache line: key, then "| tile n_buckets (dmax threads l2 ms)...".
bool read_tuned(const char* path, const std::string& key, vegas_batch* b,
                const std::vector<std::vector<Shape>>& shapes, uint64_t& tile)
{
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t bar = line.find(" | ");
        if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
        std::istringstream in(line.substr(bar + 3));
        uint64_t T = 0;
        size_t nb = 0;
        if (!(in >> T >> nb) || nb != b->buckets.size()) continue;
        if (std::find(std::begin(kTileCandidates), std::end(kTileCandidates), T) == std::end(kTileCandidates)) continue;
        std::vector<vegas_batch::Bucket> got = b->buckets;
        bool ok = true;
        for (size_t q = 0; q < nb && ok; ++q) {
            int dm = 0, th = 0, l2 = 0;
            double ms = 0.0;
            ok = bool(in >> dm >> th >> l2 >> ms) && dm == got[q].dmax;
            const Shape* hit = nullptr;
            for (const Shape& sh : shapes[q])
                if (sh.threads == th && sh.l2 == l2) hit = &sh;
            if (!ok || !hit) {
                ok = false;
                break;
            }
            apply_shape(got[q], *hit);
            got[q].tuned_ms = ms;
        }
        if (!ok) continue;
        b->buckets = got;
        tile = T;
        return true;
    }
    return false;
}

void write_tuned(const char* path, const std::string& key, const vegas_batch* b, uint64_t tile)
{
    std::ofstream f(path, std::ios::app);
    if (!f) return;  // the cache is an optimisation: a read-only place only costs the tuning
    f.precision(17);  // doubles read back exactly
    f << key << " | " << tile << " " << b->buckets.size();
    for (const auto& bk : b->buckets) f << " " << bk.dmax << " " << bk.threads << " " << bk.hrep_log2 << " " << bk.tuned_ms;
    f << "\n";
}

void destroy_graph(vegas_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

vegas_status vegas_batch_workspace_size(const vegas_desc* descs, const int64_t* n_events, int32_t n, size_t* bytes)
{
    if (!bytes) return fail(VEGAS_EINVAL, "bytes is NULL");
    vegas_status st = check_batch(descs, n_events, n);
    if (st != VEGAS_OK) return st;
    *bytes = batch_layout(descs, n_events, n).total;
    return VEGAS_OK;
}

vegas_status vegas_batch_plan(vegas_batch** out, const vegas_desc* descs, const int64_t* n_events, int32_t n,
                              void* dev_ws, size_t ws_bytes, int32_t n_iter, int32_t n_adapt, vegas_stream_t stream)
{
    if (!out) return fail(VEGAS_EINVAL, "out is NULL");
    *out = nullptr;
    vegas_status st = check_batch(descs, n_events, n);
    if (st != VEGAS_OK) return st;
    if (n_iter < 1 || n_iter > kBatchMaxIter) return fail(VEGAS_EINVAL, "n_iter must be in [1, %d]", kBatchMaxIter);
    if (n_adapt < 0 || n_adapt > n_iter) return fail(VEGAS_EINVAL, "n_adapt must be in [0, n_iter]");
    const BatchLayout L = batch_layout(descs, n_events, n);
    if (!dev_ws) return fail(VEGAS_EWORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0) return fail(VEGAS_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(VEGAS_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    vegas_batch* b = new (std::nothrow) vegas_batch();
    if (!b) return fail(VEGAS_EINVAL, "out of host memory");
    auto bail = [&](vegas_status e) {
        destroy_graph(b);
        if (b->priv) (void)hipStreamDestroy(b->priv);
        if (b->pinned) (void)hipHostFree(b->pinned);
        delete b;
        return e;
    };
    b->n = n;
    b->kind = descs[0].integrand;
    b->prec = descs[0].precision == VEGAS_FP64 ? FP64 : FP32;
    b->n_iter = n_iter;
    b->n_adapt = n_adapt;
    b->ws = dev_ws;
    b->L = L;
    int maxd = 0;
    for (int p = 0; p < n; ++p) {
        maxd = std::max(maxd, descs[p].dim);
        b->dims.push_back(descs[p].dim);
        b->bins.push_back(descs[p].n_bins);
        b->events.push_back(n_events[p]);
    }
    b->dmax = dmax_of(maxd);
    hipError_t he;
    int dev = 0, cus = 0;
    if ((he = hipStreamSynchronize(static_cast<hipStream_t>(stream))) != hipSuccess ||
        (he = hipGetDevice(&dev)) != hipSuccess ||
        (he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
        (he = hipStreamCreate(&b->priv)) != hipSuccess)
        return bail(fail(VEGAS_EHIP, "batch setup: %s", hipGetErrorString(he)));
    // one event-kernel launch per dimension bucket present; its launch shapes
    // (threads x histogram replicas that fit the LDS of the bucket's largest
    // table and histogram), optionally restricted by VEGAS_BATCH_THREADS /
    // VEGAS_BATCH_REPLICAS
    const int force_threads = env_int("VEGAS_BATCH_THREADS");
    const int force_reps = env_int("VEGAS_BATCH_REPLICAS");
    if (force_threads && force_threads != 256 && force_threads != 512 && force_threads != 1024)
        return bail(fail(VEGAS_EINVAL, "VEGAS_BATCH_THREADS must be 256, 512 or 1024"));
    if (force_reps && (force_reps < 1 || force_reps > 16 || (force_reps & (force_reps - 1))))
        return bail(fail(VEGAS_EINVAL, "VEGAS_BATCH_REPLICAS must be 1, 2, 4, 8 or 16"));
    std::vector<std::vector<Shape>> shapes;
    for (int dm : {64, 32, 16, 8, 4}) {
        // the fixed histogram layout (8 or 16 replicas) when every problem of
        // the bucket has at most kBatchFixBins bins
        bool fixable = dm <= 16;
        for (int p = 0; p < n; ++p)
            if (dmax_of(descs[p].dim) == dm && descs[p].n_bins > kBatchFixBins) fixable = false;
        auto fix_of = [&](int l2) { return fixable && (l2 == 3 || l2 == 4) ? l2 : 0; };
        auto lds_for = [&](int rep) {
            const int fl2 = fix_of(rep == 16 ? 4 : rep == 8 ? 3 : 0);
            size_t m = 0;
            for (int p = 0; p < n; ++p)
                if (dmax_of(descs[p].dim) == dm)
                    m = std::max(m, fl2 ? lds_bytes(b->prec, b->kind, descs[p].dim, descs[p].n_bins, 0)
                                        : lds_bytes(b->prec, b->kind, descs[p].dim, descs[p].n_bins, rep));
            // fixed layout: the histogram [dm][kBatchFixBins][rep] first, then the table
            return fl2 && m ? m + size_t(dm) * kBatchFixBins * rep * sizeof(double) : m;
        };
        if (lds_for(1) == 0) continue;  // no problem in this bucket
        std::vector<Shape> cand;
        for (int th : {1024, 512, 256}) {
            if (force_threads && th != force_threads) continue;
            for (int l2 = 4; l2 >= 0; --l2) {
                if (force_reps && (1 << l2) != force_reps) continue;
                const size_t lds = lds_for(1 << l2);
                // 256: the kernel's static LDS (work item, wave partials)
                if (lds + 256 > kLdsLimit) continue;
                const int bpc = batch_max_blocks_per_cu(b->prec, b->kind, dm, lds, th, fix_of(l2));
                cand.push_back(Shape{th, l2, lds, std::max(1, cus * bpc), bpc, fix_of(l2)});
            }
        }
        if (cand.empty())
            return bail(fail(VEGAS_EUNSUPPORTED, "no launch shape of the batch event kernel fits the d <= %d problems%s",
                             dm, (force_threads || force_reps) ? " (with the forced threads / replicas)" : ""));
        // starting point: the single-problem score (resident waves x a
        // replica factor, ties to the larger block)
        static const double kRepFactor[5] = {0.5, 0.65, 0.8, 0.93, 1.0};
        size_t first = 0;
        double best = -1.0;
        for (size_t c = 0; c < cand.size(); ++c) {
            const double score = double(cand[c].bpc * cand[c].threads / 64) * kRepFactor[cand[c].l2] *
                                 (cand[c].threads == 256 ? 0.92 : 1.0);
            if (score > best + 1e-9) {
                best = score;
                first = c;
            }
        }
        vegas_batch::Bucket bk;
        bk.dmax = dm;
        apply_shape(bk, cand[first]);
        b->buckets.push_back(bk);
        shapes.push_back(cand);
    }
    for (int p = 0; p < n; ++p) b->max_pstride = std::max(b->max_pstride, size_t(2 + descs[p].dim * descs[p].n_bins));
    b->pinned_bytes = std::max(sizeof(DevResult) * n, sizeof(double) * b->max_pstride) + 4096;
    if ((he = hipHostMalloc(&b->pinned, b->pinned_bytes, hipHostMallocDefault)) != hipSuccess) {
        b->pinned = nullptr;
        return bail(fail(VEGAS_EHIP, "hipHostMalloc: %s", hipGetErrorString(he)));
    }

    // per-problem state and constants
    b->probs.resize(n);
    for (int p = 0; p < n; ++p) {
        const vegas_desc& d = descs[p];
        BatchProblem& pr = b->probs[p];
        double* params = reinterpret_cast<double*>(b->at(L.params)) + size_t(p) * kMaxParams;
        DevConst* cst = reinterpret_cast<DevConst*>(b->at(L.cst)) + p;
        pr.cst = cst;
        pr.edges = reinterpret_cast<double*>(b->at(L.edges[p]));
        pr.tab64 = reinterpret_cast<double2*>(b->at(L.tab64[p]));
        pr.tab32 = reinterpret_cast<float*>(b->at(L.tab32[p]));
        pr.thr = reinterpret_cast<uint64_t*>(b->at(L.thr[p]));
        pr.last = reinterpret_cast<double*>(b->at(L.last[p]));
        pr.records = reinterpret_cast<double*>(b->at(L.records)) + size_t(p) * 2 * kBatchMaxIter;
        pr.rec_flag = reinterpret_cast<int32_t*>(b->at(L.rec_flag)) + size_t(p) * kBatchMaxIter;
        pr.result = reinterpret_cast<DevResult*>(b->at(L.results)) + p;
        pr.alpha = d.alpha;
        pr.M = double(n_events[p]);
        pr.key0 = uint32_t(d.seed);
        pr.key1 = uint32_t(d.seed >> 32);
        pr.ctr3 = uint32_t(d.problem) << 8;
        pr.d = d.dim;
        pr.N = d.n_bins;
        pr.pstride = 2 + d.dim * d.n_bins;
        if ((he = hipMemcpyAsync(params, d.params, sizeof(double) * d.n_params, hipMemcpyHostToDevice, b->priv)) !=
                hipSuccess ||
            (he = launch_prepare(b->prec, b->kind, d.dim, d.n_bins, params, cst, b->priv)) != hipSuccess)
            return bail(fail(VEGAS_EHIP, "batch prepare: %s", hipGetErrorString(he)));
    }

    // the schedule: tile size (events per work item), then each bucket's
    // launch shape, timed on this batch (or read from the tuning cache)
    const char* forced = std::getenv("VEGAS_BATCH_TILE");
    uint64_t tile = forced ? uint64_t(std::strtoull(forced, nullptr, 10)) : 0;
    if (tile && std::find(std::begin(kTileCandidates), std::end(kTileCandidates), tile) == std::end(kTileCandidates))
        return bail(fail(VEGAS_EINVAL, "VEGAS_BATCH_TILE must be one of 8192 ... 131072"));
    const bool any_forced = tile || force_threads || force_reps;
    const char* cache_path = std::getenv("VEGAS_BATCH_TUNE_CACHE");
    std::string key;
    if (cache_path && !any_forced) {
        key = tune_key(b, dev, cus);
        if (read_tuned(cache_path, key, b, shapes, tile)) b->tuned_from_cache = true;
    }
    if (!b->tuned_from_cache) {
        Timer tm;
        if ((he = tm.init(2 * int(b->buckets.size()))) != hipSuccess)
            return bail(fail(VEGAS_EHIP, "hipEventCreate: %s", hipGetErrorString(he)));
        std::vector<double> per;
        // The GPU's clock ramps up over the first tens of milliseconds of
        // sustained load, and a timing taken early reads slow.  So the
        // tuning starts with untimed runs of the starting schedule, and every
        // candidate is timed in two round-robin passes, keeping its faster
        // time: drift over the passes then touches every candidate alike.
        if ((st = upload_schedule(b, tile ? tile : kTileCandidates[2])) != VEGAS_OK) return bail(st);
        for (int w = 0; w < kTuneWarmRuns; ++w)
            if ((st = time_schedule(b, tm, per)) != VEGAS_OK) return bail(st);
        auto total = [](const std::vector<double>& v) {
            double t = 0.0;
            for (double x : v) t += x;
            return t;
        };
        if (!tile) {
            const size_t nt = sizeof(kTileCandidates) / sizeof(kTileCandidates[0]);
            std::vector<double> best_t(nt, 1e300);
            for (int pass = 0; pass < 2; ++pass)
                for (size_t c = 0; c < nt; ++c) {
                    if ((st = upload_schedule(b, kTileCandidates[c])) != VEGAS_OK) return bail(st);
                    if ((st = time_schedule(b, tm, per)) != VEGAS_OK) return bail(st);
                    best_t[c] = std::min(best_t[c], total(per));
                }
            tile = kTileCandidates[std::min_element(best_t.begin(), best_t.end()) - best_t.begin()];
        }
        if ((st = upload_schedule(b, tile)) != VEGAS_OK) return bail(st);
        // each bucket's launch is timed on its own, so the buckets are tuned
        // one after another, each keeping its fastest shape
        for (size_t q = 0; q < b->buckets.size(); ++q) {
            auto& bk = b->buckets[q];
            std::vector<double> best_s(shapes[q].size(), 1e300);
            for (int pass = 0; pass < 2; ++pass)
                for (size_t c = 0; c < shapes[q].size(); ++c) {
                    apply_shape(bk, shapes[q][c]);
                    if ((st = time_schedule(b, tm, per)) != VEGAS_OK) return bail(st);
                    best_s[c] = std::min(best_s[c], per[q]);
                }
            const size_t c = size_t(std::min_element(best_s.begin(), best_s.end()) - best_s.begin());
            apply_shape(bk, shapes[q][c]);
            bk.tuned_ms = best_s[c];
        }
        if (cache_path && !any_forced) write_tuned(cache_path, key, b, tile);
        // the timed iterations refined grids and recorded iterations: every
        // problem restarts, so the plan leaves the batch at its beginning
        if ((he = launch_batch_reset(b->args(), b->dmax, kBatchMaxIter, b->kind, b->priv)) != hipSuccess ||
            (he = hipStreamSynchronize(b->priv)) != hipSuccess)
            return bail(fail(VEGAS_EHIP, "reset after tuning: %s", hipGetErrorString(he)));
    }
    if ((st = upload_schedule(b, tile)) != VEGAS_OK) return bail(st);
    b->tuned_ms = 0.0;
    b->blocks = 0;
    for (const auto& bk : b->buckets) {
        b->blocks = std::max(b->blocks, bk.blocks);
        b->tuned_ms += bk.tuned_ms;
    }

    // record the whole run: restart, then n_iter iterations
    if ((he = hipStreamBeginCapture(b->priv, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return bail(fail(VEGAS_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(he)));
    BatchArgs a = b->args();
    vegas_status cap = VEGAS_OK;
    if ((he = launch_batch_reset(a, b->dmax, n_iter, b->kind, b->priv)) != hipSuccess)
        cap = fail(VEGAS_EHIP, "reset: %s", hipGetErrorString(he));
    for (int k = 0; k < n_iter && cap == VEGAS_OK; ++k) cap = enqueue_iteration(b, k, b->priv);
    he = hipStreamEndCapture(b->priv, &b->graph);
    if (cap != VEGAS_OK) return bail(cap);
    if (he != hipSuccess) return bail(fail(VEGAS_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(he)));
    if ((he = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
        return bail(fail(VEGAS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(he)));
    *out = b;
    return VEGAS_OK;
}

vegas_status vegas_batch_run(vegas_batch* b, vegas_stream_t stream)
{
    if (!b) return fail(VEGAS_EINVAL, "batch is NULL");
    Range r("vegas_batch_run");
    VEGAS_HIP(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
    b->next_step = 0;
    return VEGAS_OK;
}

vegas_status vegas_batch_step(vegas_batch* b, int32_t k, vegas_stream_t stream)
{
    if (!b) return fail(VEGAS_EINVAL, "batch is NULL");
    if (k < 0 || k >= b->n_iter) return fail(VEGAS_EINVAL, "iteration %d out of [0, %d)", k, b->n_iter);
    if (k != 0 && k != b->next_step)
        return fail(VEGAS_ESTATE, "iteration %d next: steps run in order from 0 (asked for %d)", b->next_step, k);
    Range r("vegas_batch_step");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (k == 0) VEGAS_HIP(launch_batch_reset(b->args(), b->dmax, b->n_iter, b->kind, s));
    vegas_status st = enqueue_iteration(b, k, s);
    if (st != VEGAS_OK) return st;
    b->next_step = k + 1 < b->n_iter ? k + 1 : 0;
    return VEGAS_OK;
}

vegas_status vegas_batch_get_iteration(vegas_batch* b, int32_t p, double* host_sums, double* host_hist,
                                       vegas_stream_t stream)
{
    if (!b) return fail(VEGAS_EINVAL, "batch is NULL");
    if (p < 0 || p >= b->n) return fail(VEGAS_EINVAL, "problem %d out of range", p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t ps = size_t(2 + b->dims[p] * b->bins[p]);
    VEGAS_HIP(hipMemcpyAsync(b->pinned, b->at(b->L.last[p]), sizeof(double) * ps, hipMemcpyDeviceToHost, s));
    VEGAS_HIP(hipStreamSynchronize(s));
    const double* v = static_cast<const double*>(b->pinned);
    if (host_sums) std::memcpy(host_sums, v, 2 * sizeof(double));
    if (host_hist) std::memcpy(host_hist, v + 2, sizeof(double) * (ps - 2));
    return VEGAS_OK;
}

vegas_status vegas_batch_results(vegas_batch* b, vegas_result_t* out, vegas_stream_t stream)
{
    if (!b || !out) return fail(VEGAS_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    VEGAS_HIP(launch_batch_combine(b->args(), b->n_iter, s));
    VEGAS_HIP(hipMemcpyAsync(b->pinned, b->at(b->L.results), sizeof(DevResult) * b->n, hipMemcpyDeviceToHost, s));
    VEGAS_HIP(hipStreamSynchronize(s));
    const DevResult* R = static_cast<const DevResult*>(b->pinned);
    int64_t bad = 0;
    for (int p = 0; p < b->n; ++p) {
        out[p].integral = R[p].integral;
        out[p].sigma = R[p].sigma;
        out[p].chi2_dof = R[p].chi2_dof;
        out[p].last_integral = R[p].last_integral;
        out[p].last_sigma = std::sqrt(R[p].last_var);
        out[p].n_iter = R[p].n_iter;
        out[p].n_combined = R[p].n_combined;
        out[p].n_events = R[p].n_events;
        out[p].n_nonfinite = R[p].n_nonfinite;
        bad += R[p].n_nonfinite;
    }
    if (bad) return fail(VEGAS_ENONFINITE, "%lld recorded iteration(s) were not finite", (long long)bad);
    return VEGAS_OK;
}

vegas_status vegas_batch_get_edges(vegas_batch* b, int32_t p, double* host, vegas_stream_t stream)
{
    if (!b || !host) return fail(VEGAS_EINVAL, "NULL argument");
    if (p < 0 || p >= b->n) return fail(VEGAS_EINVAL, "problem %d out of range", p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    VEGAS_HIP(hipMemcpyAsync(host, b->at(b->L.edges[p]), sizeof(double) * b->dims[p] * (b->bins[p] + 1),
                             hipMemcpyDeviceToHost, s));
    VEGAS_HIP(hipStreamSynchronize(s));
    return VEGAS_OK;
}

vegas_status vegas_batch_schedule(const vegas_batch* b, int64_t* tile_events, int32_t* blocks, int32_t* n_items,
                                  double* tuned_ms)
{
    if (!b) return fail(VEGAS_EINVAL, "batch is NULL");
    if (tile_events) *tile_events = int64_t(b->tile);
    if (blocks) *blocks = b->blocks;
    if (n_items) *n_items = b->n_items;
    if (tuned_ms) *tuned_ms = b->tuned_ms;
    return VEGAS_OK;
}

vegas_status vegas_batch_bucket(const vegas_batch* b, int32_t q, int32_t* n_buckets, int32_t* dmax, int32_t* threads,
                                int32_t* replicas, int32_t* blocks, double* tuned_ms, int32_t* from_cache)
{
    if (!b) return fail(VEGAS_EINVAL, "batch is NULL");
    if (n_buckets) *n_buckets = int32_t(b->buckets.size());
    if (from_cache) *from_cache = b->tuned_from_cache ? 1 : 0;
    if (q < 0) return VEGAS_OK;
    if (q >= int32_t(b->buckets.size())) return fail(VEGAS_EINVAL, "bucket %d out of range", q);
    const auto& bk = b->buckets[size_t(q)];
    if (dmax) *dmax = bk.dmax;
    if (threads) *threads = bk.threads;
    if (replicas) *replicas = 1 << bk.hrep_log2;
    if (blocks) *blocks = bk.blocks;
    if (tuned_ms) *tuned_ms = bk.tuned_ms;
    return VEGAS_OK;
}

vegas_status vegas_batch_destroy(vegas_batch* b)
{
    if (!b) return VEGAS_OK;
    destroy_graph(b);
    if (b->priv) (void)hipStreamDestroy(b->priv);
    if (b->pinned) (void)hipHostFree(b->pinned);
    delete b;
    return VEGAS_OK;
}

}  // extern "C"
