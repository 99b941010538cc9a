// C ABI of libvegas: argument validation, workspace layout, launches and the
// host-side bookkeeping of one integration context (see include/vegas.h).
#include "vegas.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "capi_util.hpp"
#include "rtc.hpp"
#include "vegas_internal.hpp"

using namespace vegas;

namespace vegas {

thread_local std::string g_err;

vegas_status fail(vegas_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

int expected_params(int kind, int d)
{
    switch (kind) {
    case VEGAS_GAUSS: return 1 + d;
    case VEGAS_BIMODAL: return 1 + 2 * d;
    case VEGAS_GENZ_DISC:
    case VEGAS_GENZ_PEAK: return 2 * d;
    }
    return -1;  // unknown, or VEGAS_USER (the caller's count)
}

vegas_status check_params(int kind, int d, const double* q)
{
    for (int k = 0; k < expected_params(kind, d); ++k)
        if (!std::isfinite(q[k])) return fail(VEGAS_EINVAL, "params[%d] is not finite", k);
    if (kind == VEGAS_GAUSS || kind == VEGAS_BIMODAL) {
        if (!(q[0] > 0.0)) return fail(VEGAS_EINVAL, "Gaussian width a must be > 0 (got %g)", q[0]);
    } else {
        for (int i = 0; i < d; ++i) {
            if (!(q[i] > 0.0)) return fail(VEGAS_EINVAL, "Genz c[%d] must be > 0 (got %g)", i, q[i]);
            if (kind == VEGAS_GENZ_DISC && !(q[d + i] >= 0.0 && q[d + i] < 1.0))
                return fail(VEGAS_EINVAL, "Genz discontinuous a[%d] must lie in [0,1) (got %g)", i, q[d + i]);
        }
    }
    return VEGAS_OK;
}

// LDS per block of the event kernel with one histogram copy per bin (the
// smallest launch it has): the grid table, the histogram and the wave
// partials of the block reduction.  Exactly what the launch asks for.
size_t event_lds_min(int prec, int kind, int d, int N)
{
    if (kind == USER) return lds_bytes(prec, USER, d, N, 1) + sizeof(double) * (kBlock / 64);
    return sample_lds(prec, kind, d, N, 1, true);
}

vegas_status check_desc(const vegas_desc* d)
{
    if (!d) return fail(VEGAS_EINVAL, "desc is NULL");
    if (d->dim < 1 || d->dim > kMaxDim) return fail(VEGAS_EINVAL, "dim must be in [1, %d] (got %d)", kMaxDim, d->dim);
    if (d->n_bins < 2 || d->n_bins > kMaxBins)
        return fail(VEGAS_EINVAL, "n_bins must be in [2, %d] (got %d)", kMaxBins, d->n_bins);
    if (d->integrand < VEGAS_GAUSS || d->integrand > VEGAS_USER)
        return fail(VEGAS_EINVAL, "unknown integrand %d", d->integrand);
    if (d->precision != VEGAS_FP64 && d->precision != VEGAS_FP32_MIXED)
        return fail(VEGAS_EINVAL, "unknown precision %d", d->precision);
    if (!(d->alpha >= 0.0) || !std::isfinite(d->alpha)) return fail(VEGAS_EINVAL, "alpha must be finite and >= 0");
    if (d->problem < 0 || d->problem >= (1 << 24)) return fail(VEGAS_EINVAL, "problem must be in [0, 2^24)");
    if (d->integrand == VEGAS_USER) {
        if (d->n_params < 0 || d->n_params > kMaxParams)
            return fail(VEGAS_EINVAL, "a user integrand takes 0..%d params (got %d)", kMaxParams, d->n_params);
        if (d->n_params > 0 && !d->params) return fail(VEGAS_EINVAL, "params is NULL");
        // the event kernel's LDS with one histogram copy: its smallest launch
        const size_t lds = event_lds_min(d->precision == VEGAS_FP64 ? FP64 : FP32, USER, d->dim, d->n_bins);
        if (lds > kLdsLimit)
            return fail(VEGAS_EUNSUPPORTED, "dim*n_bins too large: %zu bytes of LDS per block (limit %zu)", lds, kLdsLimit);
        return VEGAS_OK;
    }
    const int np = expected_params(d->integrand, d->dim);
    if (d->n_params != np) return fail(VEGAS_EINVAL, "integrand %d at dim %d takes %d params (got %d)", d->integrand, d->dim, np, d->n_params);
    if (!d->params) return fail(VEGAS_EINVAL, "params is NULL");
    const size_t lds = event_lds_min(d->precision == VEGAS_FP64 ? FP64 : FP32, d->integrand, d->dim, d->n_bins);
    if (lds > kLdsLimit)
        return fail(VEGAS_EUNSUPPORTED, "dim*n_bins too large: %zu bytes of LDS per block (limit %zu)", lds, kLdsLimit);
    return check_params(d->integrand, d->dim, d->params);
}

}  // namespace vegas

struct vegas_ctx {
    int d = 0, N = 0, kind = 0, prec = 0, problem = 0;
    uint64_t seed = 0;
    double alpha = 1.5;
    void* ws = nullptr;
    Layout L{};
    ProblemPtrs P{};
    int device = 0;
    int cu_count = 0;
    int64_t t = 0;            // next iteration index
    int rec_idx = 0;          // recorded iterations
    bool in_chunk = false;
    bool chunk_no_hist = false;  // the open iteration runs without histograms
    int64_t chunk_events = 0; // events already run in the open iteration
    bool has_hist = false;    // histograms of a finished iteration not yet refined from
    bool has_last = false;    // an iteration has finished (recorded or not)
    int64_t grid_version = 0;   // advances whenever the edges change
    int64_t params_version = 0; // advances whenever the integrand parameters change
    int blocks_user = 0;
    int blocks_auto = 0;
    int threads = kBlock;     // threads per block of the event kernel
    int hrep_log2 = 0;        // histogram replicas (log2) of the event kernel
    int hrep_user = -1;       // caller's choice (log2), -1 = automatic
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    bool timing = false;
    std::vector<hipEvent_t> tev;  // 3 per recorded call
    int n_timed = 0;
    // VEGAS_USER: the runtime-compiled module and its kernels
    int n_params = 0;
    hipModule_t umod = nullptr;
    hipFunction_t usample[2] = {nullptr, nullptr};  // with, without histograms
    hipFunction_t udump = nullptr;
    bool is_static = false;   // the per-device context of vegas_init_grid_noalloc (never freed)
};

namespace {

struct StateHeader {
    uint32_t magic, version;
    int32_t d, N, kind, prec;
    int64_t t;
    int32_t rec_idx, has_hist;
    uint64_t seed;
};
constexpr uint32_t kStateMagic = 0x56475331u;  // "VGS1"
constexpr int kTimedCalls = 1024;

void free_events(vegas_ctx* c)
{
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    c->tev.clear();
    c->n_timed = 0;
}

size_t state_bytes(const vegas_ctx* c)
{
    return sizeof(StateHeader) + sizeof(double) * c->d * (c->N + 1) + sizeof(double) * 2 * kMaxRecords +
           sizeof(int32_t) * kMaxRecords + sizeof(DevResult) + sizeof(double) * c->L.pstride;
}

int sample_blocks(const vegas_ctx* c, int64_t n)
{
    int nb = c->blocks_user > 0 ? c->blocks_user : c->blocks_auto;
    // small iterations take as many blocks as give every thread an event:
    // they are latency-bound, and a block's fixed cost (table load, histogram
    // clear and flush) runs in parallel on otherwise idle CUs (d = 4, FP64:
    // 10 iterations of 1e5 events 0.158 -> 0.106 ms against a floor of 8
    // events per thread, 3e6 events 0.244 -> 0.211 ms)
    const int64_t want = (n + int64_t(c->threads) - 1) / int64_t(c->threads);
    if (want < nb) nb = int(want);
    if (nb < 1) nb = 1;
    if (nb > kMaxBlocks) nb = kMaxBlocks;
    return nb;
}

// LDS of the runtime-compiled event kernel: table, histogram replicas, wave partials.
size_t user_lds(int prec, int d, int N, int rep, bool hist)
{
    return lds_bytes(prec, USER, d, N, hist ? rep : 0) + sizeof(double) * (kBlock / 64);
}

size_t event_lds(const vegas_ctx* c, int rep, bool hist)
{
    return c->kind == USER ? user_lds(c->prec, c->d, c->N, rep, hist) : sample_lds(c->prec, c->kind, c->d, c->N, rep, hist);
}

SampleArgs sample_args(const vegas_ctx* c, int64_t e0, int64_t n, bool no_hist)
{
    SampleArgs a{};
    a.cst = c->P.cst;
    a.tab = c->prec == FP64 ? static_cast<const void*>(c->P.tab64) : static_cast<const void*>(c->P.tab32);
    a.thr = c->P.thr;
    a.partials = c->P.partials;
    a.hslots = c->P.hslots;
    a.e0 = uint64_t(e0);
    a.n = uint64_t(n);
    a.t = uint32_t(c->t);
    a.ctr3 = uint32_t(c->problem) << 8;
    a.key0 = uint32_t(c->seed);
    a.key1 = uint32_t(c->seed >> 32);
    a.d = c->d;
    a.N = c->N;
    a.hrep_log2 = c->hrep_user >= 0 ? c->hrep_user : c->hrep_log2;
    a.hist = no_hist ? 0 : 1;
    return a;
}

MergeArgs merge_args(const vegas_ctx* c, int rows, int flags, double M)
{
    MergeArgs a{};
    a.partials = c->P.partials;
    a.hslots = c->P.hslots;
    a.acc = c->P.acc;
    a.last = c->P.last;
    a.edges = c->P.edges;
    a.tab64 = c->P.tab64;
    a.tab32 = c->P.tab32;
    a.thr = c->P.thr;
    a.cst = c->P.cst;
    a.records = c->P.records;
    a.rec_flag = c->P.rec_flag;
    a.result = c->P.result;
    a.alpha = c->alpha;
    a.M = M;
    a.rows = rows;
    a.rstride = 2;  // the rows hold S1, S2; the histogram is in hslots
    a.d = c->d;
    a.N = c->N;
    a.pstride = c->L.pstride;
    a.kind = c->kind;
    a.flags = flags;
    a.rec_idx = c->rec_idx;
    return a;
}

// The event kernel of a context: built-in, or the runtime-compiled one.
hipError_t launch_event_kernel(const vegas_ctx* c, const SampleArgs& a, int blocks, hipStream_t s)
{
    if (c->kind != USER) return launch_sample(c->prec, c->kind, a, blocks, c->threads, s);
    const bool hist = a.hist != 0;
    const double* params = c->P.params;
    void* args[] = {const_cast<SampleArgs*>(&a), const_cast<double**>(&params)};
    return hipModuleLaunchKernel(c->usample[hist ? 0 : 1], unsigned(blocks), 1, 1, unsigned(c->threads), 1, 1,
                                 unsigned(event_lds(c, 1 << a.hrep_log2, hist)), s, args, nullptr);
}

// Device-to-host copy through the pinned staging buffer, or (a context
// without one) straight into the caller's memory.
vegas_status copy_out(vegas_ctx* c, void* host, const void* dev, size_t bytes, hipStream_t s)
{
    if (!c->pinned) {
        VEGAS_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
        VEGAS_HIP(hipStreamSynchronize(s));
        return VEGAS_OK;
    }
    if (bytes > c->pinned_bytes) return fail(VEGAS_EINVAL, "internal: staging buffer too small");
    VEGAS_HIP(hipMemcpyAsync(c->pinned, dev, bytes, hipMemcpyDeviceToHost, s));
    VEGAS_HIP(hipStreamSynchronize(s));
    std::memcpy(host, c->pinned, bytes);
    return VEGAS_OK;
}

vegas_status check_edges(const double* E, int d, int N)
{
    for (int i = 0; i < d; ++i) {
        const double* e = E + size_t(i) * (N + 1);
        if (e[0] != 0.0 || e[N] != 1.0) return fail(VEGAS_EINVAL, "edges of dim %d must start at 0 and end at 1", i);
        for (int k = 0; k < N; ++k)
            if (!(e[k + 1] > e[k])) return fail(VEGAS_EINVAL, "edges of dim %d must increase strictly", i);
    }
    return VEGAS_OK;
}

}  // namespace

extern "C" {

const char* vegas_last_error(void) { return g_err.c_str(); }

vegas_status vegas_workspace_size(const vegas_desc* desc, size_t* bytes)
{
    if (!bytes) return fail(VEGAS_EINVAL, "bytes is NULL");
    vegas_status st = check_desc(desc);
    if (st != VEGAS_OK) return st;
    *bytes = make_layout(desc->dim, desc->n_bins).total;
    return VEGAS_OK;
}

}  // extern "C"

namespace {

// Context creation shared by vegas_init_grid, vegas_init_user (source: the
// user integrand's code, NULL for the built-in integrands) and
// vegas_init_grid_noalloc (into: the device's static context, filled in
// place; no host or device memory is allocated and there is no pinned
// staging buffer).
vegas_status init_ctx(vegas_ctx** out, const vegas_desc* desc, const char* source, void* dev_ws, size_t ws_bytes,
                      vegas_stream_t stream, vegas_ctx* into = nullptr)
{
    if (!out) return fail(VEGAS_EINVAL, "out is NULL");
    *out = nullptr;
    vegas_status st = check_desc(desc);
    if (st != VEGAS_OK) return st;
    if ((desc->integrand == VEGAS_USER) != (source != nullptr))
        return fail(VEGAS_EINVAL, source ? "vegas_init_user needs integrand VEGAS_USER"
                                         : "VEGAS_USER contexts are created with vegas_init_user");
    const Layout L = make_layout(desc->dim, desc->n_bins);
    if (!dev_ws) return fail(VEGAS_EWORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0) return fail(VEGAS_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(VEGAS_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    vegas_ctx* c = into;
    if (c) {
        // reused in place: timing events of an earlier use are released first
        free_events(c);
        *c = vegas_ctx();
        c->is_static = true;
    } else {
        c = new (std::nothrow) vegas_ctx();
        if (!c) return fail(VEGAS_EINVAL, "out of host memory");
    }
    c->d = desc->dim;
    c->N = desc->n_bins;
    c->kind = desc->integrand;
    c->prec = desc->precision == VEGAS_FP64 ? FP64 : FP32;
    c->problem = desc->problem;
    c->seed = desc->seed;
    c->alpha = desc->alpha;
    c->ws = dev_ws;
    c->L = L;
    c->P = problem_ptrs(dev_ws, L);
    c->n_params = desc->n_params;
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto bail = [&](vegas_status e) {
        if (c->pinned) (void)hipHostFree(c->pinned);
        if (c->umod) (void)hipModuleUnload(c->umod);
        if (c->is_static)
            *c = vegas_ctx();
        else
            delete c;
        return e;
    };
    hipError_t he;
    if ((he = hipGetDevice(&c->device)) != hipSuccess ||
        (he = hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, c->device)) != hipSuccess)
        return bail(fail(VEGAS_EHIP, "device query: %s", hipGetErrorString(he)));
    if (source) {
        std::string code, log;
        st = rtc_compile(source, c->d, c->prec, code, log);
        if (st != VEGAS_OK) return bail(st);
        if ((he = hipModuleLoadData(&c->umod, code.data())) != hipSuccess) {
            c->umod = nullptr;
            return bail(fail(VEGAS_EHIP, "hipModuleLoadData: %s", hipGetErrorString(he)));
        }
        if ((he = hipModuleGetFunction(&c->usample[0], c->umod, "vegas_user_sample")) != hipSuccess ||
            (he = hipModuleGetFunction(&c->usample[1], c->umod, "vegas_user_sample_nohist")) != hipSuccess ||
            (he = hipModuleGetFunction(&c->udump, c->umod, "vegas_user_dump")) != hipSuccess)
            return bail(fail(VEGAS_EHIP, "hipModuleGetFunction: %s", hipGetErrorString(he)));
    }
    // Launch shape of the event kernel: block size and histogram replicas.
    // Score = resident waves per CU x a replica factor x a block-size factor.
    // The factors come from the d = 8 workload on gfx950: fewer replicas leave
    // more LDS bank conflicts in the histogram atomics (4 replicas ran 17 %
    // slower than 16 at equal occupancy), and 256-thread blocks pay more
    // per-block set-up and partial rows than they gain (7 x 256 threads with
    // 4 replicas ran 11 % slower than 3 x 512 with 8 in FP64).  Ties keep the
    // larger block and the more replicas.
    // Beyond d = 8 each event makes more histogram atomics per instruction and
    // the replicas weigh more: at d = 16 (Genz, FP32-mixed) one block of 16
    // replicas ran 14 % faster than three blocks of 4 and 3 % faster than two
    // of 8, so the factors are steeper there.
    static const double kRepFactorLow[5] = {0.5, 0.65, 0.8, 0.93, 1.0};   // 1, 2, 4, 8, 16 replicas
    static const double kRepFactorHigh[5] = {0.1, 0.2, 0.35, 0.6, 1.0};
    const double* kRepFactor = c->d > 8 ? kRepFactorHigh : kRepFactorLow;
    double best = -1.0;
    int per_cu = 1;
    // 768 comes after 512, so it is taken only where it holds strictly more
    // waves (two blocks per CU where the LDS admits two and the registers
    // allow 6 or 7 waves per SIMD: the FP64 kernels up to d = 8)
    for (int th : {1024, 512, 768, 256}) {
        if (source && th > kUserThreads) continue;
        for (int l2 = 4; l2 >= 0; --l2) {
            const size_t lds = event_lds(c, 1 << l2, true);
            if (lds > kLdsLimit) continue;
            int bpc = 1;
            if (!source) {
                bpc = sample_max_blocks_per_cu(c->prec, c->kind, c->d, c->N, th, 1 << l2);
                if (bpc < 1) continue;  // beyond the kernel's largest block
            } else if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, c->usample[0], th, lds) != hipSuccess ||
                       bpc < 1) {
                bpc = 1;
            }
            const double score = double(bpc * th / 64) * kRepFactor[l2] * (th == 256 ? 0.92 : 1.0);
            if (score > best + 1e-9) {
                best = score;
                per_cu = bpc;
                c->threads = th;
                c->hrep_log2 = l2;
            }
        }
    }
    if (best < 0.0)  // check_desc admits only sizes that fit one copy; kept as a guard
        return bail(fail(VEGAS_EUNSUPPORTED, "no launch shape of the event kernel fits dim %d, n_bins %d", c->d, c->N));
    int nb = c->cu_count * per_cu;
    c->blocks_auto = nb > kMaxBlocks ? kMaxBlocks : (nb < 1 ? 1 : nb);
    if (!c->is_static) {
        c->pinned_bytes = state_bytes(c) + 4096;
        if ((he = hipHostMalloc(&c->pinned, c->pinned_bytes, hipHostMallocDefault)) != hipSuccess) {
            c->pinned = nullptr;
            return bail(fail(VEGAS_EHIP, "hipHostMalloc: %s", hipGetErrorString(he)));
        }
    }
    const size_t pbytes = sizeof(double) * desc->n_params;
    if ((pbytes > 0 && (he = hipMemcpyAsync(c->P.params, desc->params, pbytes, hipMemcpyHostToDevice, s)) != hipSuccess) ||
        (he = launch_init_state(c->P, c->d, c->N, c->L.pstride, s)) != hipSuccess ||
        (he = launch_prepare(c->prec, c->kind, c->d, c->N, c->P.params, c->P.cst, s)) != hipSuccess ||
        (he = launch_build_tables(c->P, c->kind, c->d, c->N, s)) != hipSuccess)
        return bail(fail(VEGAS_EHIP, "init: %s", hipGetErrorString(he)));
    *out = c;
    return VEGAS_OK;
}

}  // namespace

namespace vegas {

// The host half of vegas_init_grid_noalloc: a context per device, kept for the
// life of the process, over the static device workspace ws of ws_bytes.
vegas_status init_static_ctx(vegas_ctx** out, const vegas_desc* desc, int device, void* ws, size_t ws_bytes,
                             vegas_stream_t stream)
{
    static vegas_ctx g_static[kStaticDevices];
    if (device < 0 || device >= kStaticDevices)
        return fail(VEGAS_EUNSUPPORTED, "device %d: the static contexts cover devices 0..%d", device, kStaticDevices - 1);
    return init_ctx(out, desc, nullptr, ws, ws_bytes, stream, &g_static[device]);
}

}  // namespace vegas

extern "C" {

vegas_status vegas_init_grid(vegas_ctx** out, const vegas_desc* desc, void* dev_ws, size_t ws_bytes,
                             vegas_stream_t stream)
{
    return init_ctx(out, desc, nullptr, dev_ws, ws_bytes, stream);
}

vegas_status vegas_init_user(vegas_ctx** out, const vegas_desc* desc, const char* source, void* dev_ws,
                             size_t ws_bytes, vegas_stream_t stream)
{
    if (!source) {
        if (out) *out = nullptr;
        return fail(VEGAS_EINVAL, "source is NULL");
    }
    return init_ctx(out, desc, source, dev_ws, ws_bytes, stream);
}

vegas_status vegas_user_compile(const char* source, int32_t dim, int32_t precision, char* log, size_t log_bytes)
{
    if (!source) return fail(VEGAS_EINVAL, "source is NULL");
    if (dim < 1 || dim > kMaxDim) return fail(VEGAS_EINVAL, "dim must be in [1, %d] (got %d)", kMaxDim, dim);
    if (precision != VEGAS_FP64 && precision != VEGAS_FP32_MIXED)
        return fail(VEGAS_EINVAL, "unknown precision %d", precision);
    std::string code, msg;
    const vegas_status st = rtc_compile(source, dim, precision == VEGAS_FP64 ? FP64 : FP32, code, msg);
    if (log && log_bytes > 0) {
        const size_t n = std::min(msg.size(), log_bytes - 1);
        std::memcpy(log, msg.data(), n);
        log[n] = '\0';
    }
    return st;
}

}  // extern "C"

namespace {

// vegas_iterate, and with dev_G (vegas_iterate_grad) the forward pass that
// also forms the estimate's gradient into dev_G; dev_out2 (optional): the
// reduction also writes (I_t, sigma_t) there.
vegas_status iterate_impl(vegas_ctx* c, int64_t n, uint32_t flags, double* dev_G, double* dev_out2,
                          vegas_stream_t stream)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (n < 1 || n > (int64_t(1) << 40)) return fail(VEGAS_EINVAL, "n_events must be in [1, 2^40] (got %lld)", (long long)n);
    if (flags & ~uint32_t(VEGAS_CHUNK_BEGIN | VEGAS_CHUNK_END | VEGAS_NO_COMBINE | VEGAS_REFINE | VEGAS_NO_HIST |
                          VEGAS_NO_RECORD))
        return fail(VEGAS_EINVAL, "unknown flags 0x%x", flags);
    const bool begin = flags & VEGAS_CHUNK_BEGIN, end = flags & VEGAS_CHUNK_END;
    const bool no_hist = flags & VEGAS_NO_HIST;
    const bool no_record = flags & VEGAS_NO_RECORD;
    if ((flags & (VEGAS_NO_COMBINE | VEGAS_REFINE | VEGAS_NO_RECORD)) && !end)
        return fail(VEGAS_EINVAL, "REFINE / NO_COMBINE / NO_RECORD only apply with CHUNK_END");
    if (no_hist && (flags & VEGAS_REFINE)) return fail(VEGAS_EINVAL, "REFINE needs the histograms (NO_HIST given)");
    if (begin && c->in_chunk) return fail(VEGAS_ESTATE, "CHUNK_BEGIN while an iteration is open");
    if (!begin && !c->in_chunk) return fail(VEGAS_ESTATE, "no open iteration: start with CHUNK_BEGIN");
    if (!begin && no_hist != c->chunk_no_hist)
        return fail(VEGAS_EINVAL, "NO_HIST must be given on every chunk of an iteration or on none");
    const int64_t e0 = begin ? 0 : c->chunk_events;
    const int64_t M = e0 + n;
    if (M > (int64_t(1) << 40)) return fail(VEGAS_EINVAL, "iteration exceeds 2^40 events");
    if (end && M < 2) return fail(VEGAS_EINVAL, "an iteration needs at least 2 events");
    if (end && !no_record && c->rec_idx >= kMaxRecords)
        return fail(VEGAS_ESTATE, "%d iterations recorded: call vegas_reset_results", kMaxRecords);
    if (c->t >= (int64_t(1) << 32)) return fail(VEGAS_ESTATE, "iteration index exhausted");

    if (dev_G) {
        if (c->kind != VEGAS_GAUSS) return fail(VEGAS_EUNSUPPORTED, "the gradient is implemented for the Gaussian integrand");
        if (!begin || !end || !no_hist)
            return fail(VEGAS_EINVAL, "the forward pass with the gradient is one whole iteration without histograms "
                                      "(VEGAS_ITER_FULL | VEGAS_NO_HIST)");
    }

    hipStream_t s = static_cast<hipStream_t>(stream);
    const int blocks = sample_blocks(c, n);
    const SampleArgs a = sample_args(c, e0, n, no_hist);
    const bool timed = c->timing && c->n_timed < kTimedCalls;
    if (timed) VEGAS_HIP(hipEventRecord(c->tev[3 * c->n_timed], s));
    if (dev_G)
        VEGAS_HIP(launch_sample_grad(c->prec, a, c->P.adj_part, blocks, c->threads, s));
    else
        VEGAS_HIP(launch_event_kernel(c, a, blocks, s));
    if (timed) VEGAS_HIP(hipEventRecord(c->tev[3 * c->n_timed + 1], s));
    int mf = (begin ? MERGE_BEGIN : 0) | (end ? MERGE_END : 0) | ((flags & VEGAS_NO_COMBINE) ? MERGE_NO_COMBINE : 0) |
             ((flags & VEGAS_REFINE) ? MERGE_REFINE : 0) | (no_hist ? MERGE_NO_HIST : 0) |
             (no_record ? MERGE_NO_RECORD : 0) | (dev_G ? MERGE_GRAD : 0);
    MergeArgs ma = merge_args(c, blocks, mf, double(M));
    ma.gpart = c->P.adj_part;
    ma.grad_out = dev_G;
    ma.last_out = dev_out2;
    VEGAS_HIP(launch_merge(ma, s));
    if (timed) {
        VEGAS_HIP(hipEventRecord(c->tev[3 * c->n_timed + 2], s));
        c->n_timed += 1;
    }

    c->chunk_events = M;
    c->in_chunk = !end;
    c->chunk_no_hist = no_hist;
    if (end) {
        c->t += 1;
        if (!no_record) c->rec_idx += 1;
        c->has_hist = !(flags & VEGAS_REFINE) && !no_hist;
        c->has_last = true;
        if (flags & VEGAS_REFINE) c->grid_version += 1;
        c->chunk_events = 0;
    }
    return VEGAS_OK;
}

}  // namespace

extern "C" {

vegas_status vegas_iterate(vegas_ctx* c, int64_t n, uint32_t flags, vegas_stream_t stream)
{
    Range r("vegas_iterate");
    return iterate_impl(c, n, flags, nullptr, nullptr, stream);
}

vegas_status vegas_iterate_grad(vegas_ctx* c, int64_t n, uint32_t flags, double* dev_G, vegas_stream_t stream)
{
    if (!dev_G) return fail(VEGAS_EINVAL, "dev_G is NULL");
    Range r("vegas_iterate_grad");
    return iterate_impl(c, n, flags, dev_G, nullptr, stream);
}

vegas_status vegas_forward_grad(vegas_ctx* c, const void* dev_params, const void* dev_params_rest, int32_t n_params,
                                int32_t is_fp32, int64_t n, uint32_t flags, double* dev_G, double* dev_out2,
                                vegas_stream_t stream)
{
    if (!c || !dev_params || !dev_G || !dev_out2) return fail(VEGAS_EINVAL, "NULL argument");
    Range r("vegas_forward_grad");
    if (c->kind != VEGAS_GAUSS) return fail(VEGAS_EUNSUPPORTED, "the gradient is implemented for the Gaussian integrand");
    if (n_params != expected_params(c->kind, c->d)) return fail(VEGAS_EINVAL, "expected %d params, got %d",
                                                               expected_params(c->kind, c->d), n_params);
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    // the iteration's checks first, so that a refused call changes nothing
    if (n < 2 || n > (int64_t(1) << 40)) return fail(VEGAS_EINVAL, "n_events must be in [2, 2^40]");
    if ((flags & (VEGAS_ITER_FULL | VEGAS_NO_HIST)) != (VEGAS_ITER_FULL | VEGAS_NO_HIST) ||
        (flags & ~uint32_t(VEGAS_ITER_FULL | VEGAS_NO_HIST | VEGAS_NO_COMBINE | VEGAS_NO_RECORD)))
        return fail(VEGAS_EINVAL, "flags must be VEGAS_ITER_FULL | VEGAS_NO_HIST, optionally with NO_COMBINE, NO_RECORD");
    if (!(flags & VEGAS_NO_RECORD) && c->rec_idx >= kMaxRecords)
        return fail(VEGAS_ESTATE, "%d iterations recorded: call vegas_reset_results", kMaxRecords);
    if (c->t >= (int64_t(1) << 32)) return fail(VEGAS_ESTATE, "iteration index exhausted");
    VEGAS_HIP(launch_set_params(c->prec, c->kind, c->d, c->N, dev_params, n_params, is_fp32 ? 1 : 0, c->P,
                                static_cast<hipStream_t>(stream), dev_params_rest));
    c->params_version += 1;
    return iterate_impl(c, n, flags, dev_G, dev_out2, stream);
}

vegas_status vegas_grad_scale(const double* dev_G, const double* dev_gout, void* dev_grad, int32_t n,
                              int32_t grad_fp32, vegas_stream_t stream)
{
    if (!dev_G || !dev_gout || !dev_grad) return fail(VEGAS_EINVAL, "NULL argument");
    if (n < 1 || n > kMaxDim + 1) return fail(VEGAS_EINVAL, "n must be in [1, %d]", kMaxDim + 1);
    VEGAS_HIP(launch_grad_scale(dev_G, dev_gout, dev_grad, n, grad_fp32 ? 1 : 0, static_cast<hipStream_t>(stream)));
    return VEGAS_OK;
}

vegas_status vegas_time_event_kernel(vegas_ctx* c, int64_t n, int32_t reps, int32_t no_hist, double* ms,
                                     vegas_stream_t stream)
{
    if (!c || !ms) return fail(VEGAS_EINVAL, "NULL argument");
    if (n < 1 || n > (int64_t(1) << 40)) return fail(VEGAS_EINVAL, "n_events must be in [1, 2^40]");
    if (reps < 1 || reps > 10000) return fail(VEGAS_EINVAL, "reps must be in [1, 10000]");
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int blocks = sample_blocks(c, n);
    const SampleArgs a = sample_args(c, 0, n, no_hist != 0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    for (int r = 0; r < reps && he == hipSuccess; ++r) he = launch_event_kernel(c, a, blocks, s);
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    // the launches added into the histogram accumulators: clear them
    if (he == hipSuccess) he = launch_zero(c->P.hslots, size_t(kHistSlots) * c->d * c->N, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float el = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&el, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (he != hipSuccess) return fail(VEGAS_EHIP, "time_event_kernel: %s", hipGetErrorString(he));
    *ms = double(el) / reps;
    return VEGAS_OK;
}

vegas_status vegas_refine(vegas_ctx* c, vegas_stream_t stream)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    if (!c->has_hist) return fail(VEGAS_ESTATE, "no completed iteration whose histograms are unused");
    Range r("vegas_refine");
    VEGAS_HIP(launch_refine(merge_args(c, 1, 0, 0.0), static_cast<hipStream_t>(stream)));
    c->has_hist = false;
    c->grid_version += 1;
    return VEGAS_OK;
}

vegas_status vegas_result(vegas_ctx* c, vegas_result_t* out, vegas_stream_t stream)
{
    if (!c || !out) return fail(VEGAS_EINVAL, "NULL argument");
    Range r("vegas_result");
    DevResult R;
    hipStream_t s = static_cast<hipStream_t>(stream);
    VEGAS_HIP(launch_combine(c->P.records, c->P.rec_flag, c->rec_idx, c->P.result, s));
    vegas_status st = copy_out(c, &R, c->P.result, sizeof(R), s);
    if (st != VEGAS_OK) return st;
    out->integral = R.integral;
    out->sigma = R.sigma;
    out->chi2_dof = R.chi2_dof;
    out->last_integral = R.last_integral;
    out->last_sigma = std::sqrt(R.last_var);
    out->n_iter = R.n_iter;
    out->n_combined = R.n_combined;
    out->n_events = R.n_events;
    out->n_nonfinite = R.n_nonfinite;
    if (R.n_nonfinite > 0) return fail(VEGAS_ENONFINITE, "%lld recorded iteration(s) were not finite", (long long)R.n_nonfinite);
    return VEGAS_OK;
}

vegas_status vegas_reset_results(vegas_ctx* c, vegas_stream_t stream)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    VEGAS_HIP(launch_reset_results(c->P.records, c->P.rec_flag, c->P.result, static_cast<hipStream_t>(stream)));
    c->rec_idx = 0;
    return VEGAS_OK;
}

vegas_status vegas_set_params_device(vegas_ctx* c, const void* dev_params, int32_t n, int32_t is_fp32,
                                     vegas_stream_t stream)
{
    if (!c || !dev_params) return fail(VEGAS_EINVAL, "NULL argument");
    const int want = c->kind == USER ? c->n_params : expected_params(c->kind, c->d);
    if (n != want) return fail(VEGAS_EINVAL, "expected %d params, got %d", want, n);
    if (n == 0) return VEGAS_OK;
    // parameters, derived constants and the tables (FP32 entries are offsets
    // from the centres) in one launch
    VEGAS_HIP(launch_set_params(c->prec, c->kind, c->d, c->N, dev_params, n, is_fp32 ? 1 : 0, c->P,
                                static_cast<hipStream_t>(stream)));
    c->params_version += 1;
    return VEGAS_OK;
}

vegas_status vegas_get_params_device(vegas_ctx* c, double* dev_out, vegas_stream_t stream)
{
    if (!c || !dev_out) return fail(VEGAS_EINVAL, "NULL argument");
    const int n = c->kind == USER ? c->n_params : expected_params(c->kind, c->d);
    if (n == 0) return VEGAS_OK;
    VEGAS_HIP(hipMemcpyAsync(dev_out, c->P.params, sizeof(double) * n, hipMemcpyDeviceToDevice,
                             static_cast<hipStream_t>(stream)));
    return VEGAS_OK;
}

vegas_status vegas_get_versions(const vegas_ctx* c, int64_t* grid_version, int64_t* params_version)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (grid_version) *grid_version = c->grid_version;
    if (params_version) *params_version = c->params_version;
    return VEGAS_OK;
}

vegas_status vegas_last_iteration_device(vegas_ctx* c, double* dev_out, vegas_stream_t stream)
{
    if (!c || !dev_out) return fail(VEGAS_EINVAL, "NULL argument");
    if (!c->has_last && c->rec_idx == 0) return fail(VEGAS_ESTATE, "no finished iteration");
    VEGAS_HIP(launch_copy_last(c->P.result, dev_out, static_cast<hipStream_t>(stream)));
    return VEGAS_OK;
}

vegas_status vegas_adjoint(vegas_ctx* c, int64_t iteration, int64_t n, const double* dev_gout, void* dev_grad,
                           int32_t grad_fp32, vegas_stream_t stream)
{
    if (!c || !dev_gout || !dev_grad) return fail(VEGAS_EINVAL, "NULL argument");
    if (c->kind != VEGAS_GAUSS) return fail(VEGAS_EUNSUPPORTED, "the adjoint is implemented for the Gaussian integrand");
    if (iteration < 0 || iteration >= (int64_t(1) << 32)) return fail(VEGAS_EINVAL, "iteration out of range");
    if (n < 1 || n > (int64_t(1) << 40)) return fail(VEGAS_EINVAL, "n_events must be in [1, 2^40]");
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    Range r("vegas_adjoint");
    AdjointArgs a{};
    a.cst = c->P.cst;
    a.tab = c->prec == FP64 ? static_cast<const void*>(c->P.tab64) : static_cast<const void*>(c->P.tab32);
    a.partials = c->P.adj_part;
    a.gout = dev_gout;
    a.grad = dev_grad;
    a.n = uint64_t(n);
    a.t = uint32_t(iteration);
    a.ctr3 = uint32_t(c->problem) << 8;
    a.key0 = uint32_t(c->seed);
    a.key1 = uint32_t(c->seed >> 32);
    a.d = c->d;
    a.N = c->N;
    a.grad_fp32 = grad_fp32 ? 1 : 0;
    VEGAS_HIP(launch_adjoint(c->prec, a, sample_blocks(c, n), static_cast<hipStream_t>(stream)));
    return VEGAS_OK;
}

vegas_status vegas_dump_events(vegas_ctx* c, int64_t iteration, int64_t first, int64_t count, double* dev_out,
                               vegas_stream_t stream)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (iteration < 0 || iteration >= (int64_t(1) << 32)) return fail(VEGAS_EINVAL, "iteration out of range");
    if (first < 0 || count < 0 || first + count > (int64_t(1) << 40)) return fail(VEGAS_EINVAL, "event range out of bounds");
    if (count == 0) return VEGAS_OK;
    if (!dev_out) return fail(VEGAS_EINVAL, "dev_out is NULL");
    DumpArgs a{};
    a.cst = c->P.cst;
    a.tab = c->prec == FP64 ? static_cast<const void*>(c->P.tab64) : static_cast<const void*>(c->P.tab32);
    a.thr = c->P.thr;
    a.out = dev_out;
    a.e0 = uint64_t(first);
    a.n = uint64_t(count);
    a.t = uint32_t(iteration);
    a.ctr3 = uint32_t(c->problem) << 8;
    a.key0 = uint32_t(c->seed);
    a.key1 = uint32_t(c->seed >> 32);
    a.d = c->d;
    a.N = c->N;
    if (c->kind == USER) {
        // one event per thread, 256 threads, the table in LDS
        const uint64_t blocks = std::min<uint64_t>((a.n + 255) / 256, 4096);
        const double* params = c->P.params;
        void* args[] = {&a, const_cast<double**>(&params)};
        VEGAS_HIP(hipModuleLaunchKernel(c->udump, unsigned(blocks), 1, 1, 256, 1, 1,
                                        unsigned(tab_entry_bytes(c->prec, USER) * c->d * c->N),
                                        static_cast<hipStream_t>(stream), args, nullptr));
        return VEGAS_OK;
    }
    VEGAS_HIP(launch_dump(c->prec, c->kind, a, static_cast<hipStream_t>(stream)));
    return VEGAS_OK;
}

vegas_status vegas_get_edges(vegas_ctx* c, double* host, vegas_stream_t stream)
{
    if (!c || !host) return fail(VEGAS_EINVAL, "NULL argument");
    return copy_out(c, host, c->P.edges, sizeof(double) * c->d * (c->N + 1), static_cast<hipStream_t>(stream));
}

vegas_status vegas_set_edges(vegas_ctx* c, const double* host, vegas_stream_t stream)
{
    if (!c || !host) return fail(VEGAS_EINVAL, "NULL argument");
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    vegas_status st = check_edges(host, c->d, c->N);
    if (st != VEGAS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    VEGAS_HIP(hipMemcpyAsync(c->P.edges, host, sizeof(double) * c->d * (c->N + 1), hipMemcpyHostToDevice, s));
    VEGAS_HIP(launch_build_tables(c->P, c->kind, c->d, c->N, s));
    c->grid_version += 1;
    return VEGAS_OK;
}

vegas_status vegas_get_iteration(vegas_ctx* c, double* sums, double* hist, vegas_stream_t stream)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (c->rec_idx == 0 && !c->has_hist) return fail(VEGAS_ESTATE, "no completed iteration");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!c->pinned) {
        if (sums) VEGAS_HIP(hipMemcpyAsync(sums, c->P.last, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (hist)
            VEGAS_HIP(hipMemcpyAsync(hist, c->P.last + 2, sizeof(double) * c->d * c->N, hipMemcpyDeviceToHost, s));
        VEGAS_HIP(hipStreamSynchronize(s));
        return VEGAS_OK;
    }
    const size_t bytes = sizeof(double) * c->L.pstride;
    if (bytes > c->pinned_bytes) return fail(VEGAS_EINVAL, "internal: staging buffer too small");
    VEGAS_HIP(hipMemcpyAsync(c->pinned, c->P.last, bytes, hipMemcpyDeviceToHost, s));
    VEGAS_HIP(hipStreamSynchronize(s));
    const double* v = static_cast<const double*>(c->pinned);
    if (sums) std::memcpy(sums, v, 2 * sizeof(double));
    if (hist) std::memcpy(hist, v + 2, sizeof(double) * c->d * c->N);
    return VEGAS_OK;
}

vegas_status vegas_state_size(const vegas_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return fail(VEGAS_EINVAL, "NULL argument");
    *bytes = state_bytes(c);
    return VEGAS_OK;
}

vegas_status vegas_get_state(vegas_ctx* c, void* host_buf, size_t bytes, vegas_stream_t stream)
{
    if (!c || !host_buf) return fail(VEGAS_EINVAL, "NULL argument");
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    if (bytes < state_bytes(c)) return fail(VEGAS_EINVAL, "state buffer has %zu bytes, needs %zu", bytes, state_bytes(c));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // staged through the pinned buffer, or copied straight into host_buf
    char* p = c->pinned ? static_cast<char*>(c->pinned) : static_cast<char*>(host_buf);
    StateHeader h{kStateMagic, 1u, c->d, c->N, c->kind, c->prec, c->t, c->rec_idx, c->has_hist ? 1 : 0, c->seed};
    std::memcpy(p, &h, sizeof(h));
    size_t o = sizeof(h);
    const size_t eb = sizeof(double) * c->d * (c->N + 1), rb = sizeof(double) * 2 * kMaxRecords,
                 fb = sizeof(int32_t) * kMaxRecords, lb = sizeof(double) * c->L.pstride;
    VEGAS_HIP(launch_combine(c->P.records, c->P.rec_flag, c->rec_idx, c->P.result, s));
    VEGAS_HIP(hipMemcpyAsync(p + o, c->P.edges, eb, hipMemcpyDeviceToHost, s));
    o += eb;
    VEGAS_HIP(hipMemcpyAsync(p + o, c->P.records, rb, hipMemcpyDeviceToHost, s));
    o += rb;
    VEGAS_HIP(hipMemcpyAsync(p + o, c->P.rec_flag, fb, hipMemcpyDeviceToHost, s));
    o += fb;
    VEGAS_HIP(hipMemcpyAsync(p + o, c->P.result, sizeof(DevResult), hipMemcpyDeviceToHost, s));
    o += sizeof(DevResult);
    VEGAS_HIP(hipMemcpyAsync(p + o, c->P.last, lb, hipMemcpyDeviceToHost, s));
    o += lb;
    VEGAS_HIP(hipStreamSynchronize(s));
    if (p != host_buf) std::memcpy(host_buf, p, o);
    return VEGAS_OK;
}

vegas_status vegas_set_state(vegas_ctx* c, const void* host_buf, size_t bytes, vegas_stream_t stream)
{
    if (!c || !host_buf) return fail(VEGAS_EINVAL, "NULL argument");
    if (c->in_chunk) return fail(VEGAS_ESTATE, "an iteration is open");
    if (bytes < state_bytes(c)) return fail(VEGAS_EINVAL, "state buffer has %zu bytes, needs %zu", bytes, state_bytes(c));
    StateHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (h.magic != kStateMagic || h.version != 1u) return fail(VEGAS_EINVAL, "not a vegas state");
    if (h.d != c->d || h.N != c->N || h.kind != c->kind || h.prec != c->prec || h.seed != c->seed)
        return fail(VEGAS_EINVAL, "state belongs to a different problem");
    if (h.rec_idx < 0 || h.rec_idx > kMaxRecords || h.t < 0) return fail(VEGAS_EINVAL, "corrupt state");
    const char* p = static_cast<const char*>(host_buf) + sizeof(h);
    if (check_edges(reinterpret_cast<const double*>(p), c->d, c->N) != VEGAS_OK) return VEGAS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t eb = sizeof(double) * c->d * (c->N + 1), rb = sizeof(double) * 2 * kMaxRecords,
                 fb = sizeof(int32_t) * kMaxRecords, lb = sizeof(double) * c->L.pstride;
    VEGAS_HIP(hipMemcpyAsync(c->P.edges, p, eb, hipMemcpyHostToDevice, s));
    p += eb;
    VEGAS_HIP(hipMemcpyAsync(c->P.records, p, rb, hipMemcpyHostToDevice, s));
    p += rb;
    VEGAS_HIP(hipMemcpyAsync(c->P.rec_flag, p, fb, hipMemcpyHostToDevice, s));
    p += fb;
    VEGAS_HIP(hipMemcpyAsync(c->P.result, p, sizeof(DevResult), hipMemcpyHostToDevice, s));
    p += sizeof(DevResult);
    VEGAS_HIP(hipMemcpyAsync(c->P.last, p, lb, hipMemcpyHostToDevice, s));
    VEGAS_HIP(launch_build_tables(c->P, c->kind, c->d, c->N, s));
    c->t = h.t;
    c->rec_idx = h.rec_idx;
    c->has_hist = h.has_hist != 0;
    c->has_last = h.rec_idx > 0;
    c->grid_version += 1;
    return VEGAS_OK;
}

vegas_status vegas_get_iteration_index(const vegas_ctx* c, int64_t* t)
{
    if (!c || !t) return fail(VEGAS_EINVAL, "NULL argument");
    *t = c->t;
    return VEGAS_OK;
}

vegas_status vegas_set_launch(vegas_ctx* c, int32_t n_blocks)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (n_blocks < 0 || n_blocks > kMaxBlocks) return fail(VEGAS_EINVAL, "n_blocks must be in [0, %d]", kMaxBlocks);
    c->blocks_user = n_blocks;
    return VEGAS_OK;
}

vegas_status vegas_set_hist_replicas(vegas_ctx* c, int32_t replicas)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (replicas == 0) {
        c->hrep_user = -1;
        return VEGAS_OK;
    }
    int l2 = 0;
    while ((1 << l2) < replicas) ++l2;
    if (replicas < 0 || (1 << l2) != replicas || l2 > 4)
        return fail(VEGAS_EINVAL, "replicas must be 0 (automatic) or 1, 2, 4, 8, 16");
    const size_t lds = event_lds(c, replicas, true);
    if (lds > kLdsLimit) return fail(VEGAS_EUNSUPPORTED, "%d replicas need %zu bytes of LDS", replicas, lds);
    c->hrep_user = l2;
    return VEGAS_OK;
}

vegas_status vegas_get_launch(const vegas_ctx* c, int32_t* auto_blocks, int32_t* blocks_per_cu, int32_t* threads,
                              int32_t* replicas)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (auto_blocks) *auto_blocks = c->blocks_auto;
    if (blocks_per_cu) *blocks_per_cu = c->cu_count > 0 ? c->blocks_auto / c->cu_count : 0;
    if (threads) *threads = c->threads;
    if (replicas) *replicas = 1 << (c->hrep_user >= 0 ? c->hrep_user : c->hrep_log2);
    return VEGAS_OK;
}

vegas_status vegas_timing_enable(vegas_ctx* c, int32_t enable)
{
    if (!c) return fail(VEGAS_EINVAL, "ctx is NULL");
    if (enable && c->tev.empty()) {
        c->tev.resize(3 * kTimedCalls);
        for (auto& e : c->tev) {
            hipError_t he = hipEventCreate(&e);
            if (he != hipSuccess) {
                e = nullptr;
                c->tev.erase(std::remove(c->tev.begin(), c->tev.end(), nullptr), c->tev.end());
                free_events(c);
                return fail(VEGAS_EHIP, "hipEventCreate: %s", hipGetErrorString(he));
            }
        }
    }
    c->timing = enable != 0;
    c->n_timed = 0;
    return VEGAS_OK;
}

vegas_status vegas_timing_read(vegas_ctx* c, double* sample_ms, double* merge_ms, int64_t* count)
{
    if (!c || !sample_ms || !merge_ms || !count) return fail(VEGAS_EINVAL, "NULL argument");
    double ts = 0.0, tm = 0.0;
    if (c->n_timed > 0) {
        VEGAS_HIP(hipEventSynchronize(c->tev[3 * (c->n_timed - 1) + 2]));
        for (int k = 0; k < c->n_timed; ++k) {
            float a = 0.f, b = 0.f;
            VEGAS_HIP(hipEventElapsedTime(&a, c->tev[3 * k], c->tev[3 * k + 1]));
            VEGAS_HIP(hipEventElapsedTime(&b, c->tev[3 * k + 1], c->tev[3 * k + 2]));
            ts += a;
            tm += b;
        }
    }
    *sample_ms = ts;
    *merge_ms = tm;
    *count = c->n_timed;
    c->n_timed = 0;
    return VEGAS_OK;
}

vegas_status vegas_destroy(vegas_ctx* c)
{
    if (!c) return VEGAS_OK;
    if (c->is_static) return VEGAS_OK;  // the device's static context lives on
    free_events(c);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->umod) (void)hipModuleUnload(c->umod);
    delete c;
    return VEGAS_OK;
}

}  // extern "C"
