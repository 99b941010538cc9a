// Internal declarations shared by the HIP kernels and the C-ABI host code.
// The device part is also handed to the runtime compiler for user integrands
// (__HIPCC_RTC__ defined): there the HIP device API is built in and only the
// fixed-width integer names are missing.
#pragma once

#ifdef __HIPCC_RTC__
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::uint64_t uint64_t;
#else
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#endif

namespace vegas {

constexpr int kMaxDim = 64;
constexpr int kMaxBins = 255;
constexpr int kMaxParams = 1 + 2 * kMaxDim;
constexpr int kMaxRecords = 1024;   // recorded iterations per context
constexpr int kBlock = 1024;        // threads per block of the event kernels
constexpr int kMaxBlocks = 2048;    // rows of the per-block partial table
// The event kernel adds each block's histogram into slot ((block / 8) mod
// kHistSlots) with device-scope atomics; the reduction adds the slots.
constexpr int kHistSlots = 8;
constexpr int kMergeThreads = 1024; // threads per block of the reduction kernel
constexpr size_t kLdsLimit = 160 * 1024;

// USER: an integrand compiled at run time from the caller's source
enum Kind { GAUSS = 0, BIMODAL = 1, GENZ_DISC = 2, GENZ_PEAK = 3, USER = 4 };
enum Prec { FP64 = 0, FP32 = 1 };

// Derived per-problem constants, computed on the device from the raw FP64
// parameters whenever they change.  The event kernels compute
//   F  = the integrand's significand in the kernel precision,
//   wp = product of the bin widths (FP32: each scaled by 2^ws, ws = round(log2 N)),
// and the event value v = f w = 2^(ew + fe) (F * wp) * C with C = Cf * Cw,
// Cf the integrand normalisation and Cw = N^d (FP32: N^d 2^(-ws d)).
struct DevConst {
    double C;        // Cf * Cw
    double Cf;       // f = 2^fe F Cf
    double Cw;       // w = 2^ew wp Cw
    double kexp64;   // GAUSS, BIMODAL: 1/a^2
    double kexp2_64; // GAUSS, BIMODAL: log2(e)/a^2; DISC: log2(e)
    double inv_a;    // GAUSS, BIMODAL: 1/a (adjoint)
    int32_t n_bins;  // N (binning)
    int32_t pad1;
    double two_m32;  // 2^-32
    float kexp32;    // (unused by the kernels; kept for the layout)
    float dscale32;  // 2^-ws
    float ka32;      // GAUSS: RN32(1/a^2) (adjoint)
    float pad0;
    double p1_64[kMaxDim];  // GAUSS mu | BIMODAL muA | DISC c | PEAK c^2
    double p2_64[kMaxDim];  //          | BIMODAL muB - muA | DISC a | PEAK a
    float p1_32[kMaxDim];   // PEAK c^2
    float p2_32[kMaxDim];   // (unused)
    double cA64[kMaxDim];   // table centres: GAUSS mu | BIMODAL muA | DISC, PEAK a
    double cB64[kMaxDim];   // BIMODAL muB
};

// Result block kept on the device; mirrors vegas_result_t plus the last variance.
struct DevResult {
    double integral, sigma, chi2_dof, last_integral, last_var;
    int64_t n_iter, n_combined, n_events, n_nonfinite;
};

// Byte offsets of the regions of a single-problem workspace.
struct Layout {
    size_t params;    // double[kMaxParams]
    size_t cst;       // DevConst
    size_t edges;     // double[d][N+1]
    size_t tab64;     // double2[d][N]  (E_b, E_{b+1}-E_b)
    size_t tab32;     // float2 or float4 [d][N]  (offsets from the centres, scaled width)
    size_t thr;       // uint64[d]  Genz discontinuous: x_i > a_i as an integer threshold
    size_t partials;  // double[kMaxBlocks][2]  per-block (S1, S2) of the event kernel
    size_t hslots;    // double[kHistSlots][d*N]  histogram accumulators of the event kernel
    size_t acc;       // double[2][pstride]   chunk accumulators (hi, lo)
    size_t last;      // double[pstride]      S1, S2, H of the last completed iteration
    size_t records;   // double[kMaxRecords][2]  (I_t, var_t)
    size_t rec_flag;  // int32[kMaxRecords]      combined?
    size_t result;    // DevResult
    size_t adj_part;  // double[kMaxBlocks][kMaxDim + 1]
    size_t total;
    int pstride;      // 2 + d*N
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout make_layout(int d, int N)
{
    Layout L{};
    const int ps = 2 + d * N;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.params = take(sizeof(double) * kMaxParams);
    L.cst = take(sizeof(DevConst));
    L.edges = take(sizeof(double) * d * (N + 1));
    L.tab64 = take(sizeof(double) * 2 * d * N);
    L.tab32 = take(sizeof(float) * 4 * d * N);
    L.thr = take(sizeof(uint64_t) * d);
    L.partials = take(sizeof(double) * size_t(kMaxBlocks) * 2);
    L.hslots = take(sizeof(double) * size_t(kHistSlots) * d * N);
    L.acc = take(sizeof(double) * 2 * size_t(ps));
    L.last = take(sizeof(double) * size_t(ps));
    L.records = take(sizeof(double) * 2 * kMaxRecords);
    L.rec_flag = take(sizeof(int32_t) * kMaxRecords);
    L.result = take(sizeof(DevResult));
    L.adj_part = take(sizeof(double) * size_t(kMaxBlocks) * (kMaxDim + 1));
    L.total = o;
    L.pstride = ps;
    return L;
}

// Bytes of one grid-table entry in LDS.
inline size_t tab_entry_bytes(int prec, int kind)
{
    return prec == FP64 ? 16 : (kind == BIMODAL ? 16 : 8);
}

// LDS of the event kernel: grid table, then the histogram with `rep`
// replicas per bin ([dim][bin][replica]; lane l adds into replica l mod rep).
inline size_t lds_bytes(int prec, int kind, int d, int N, int rep = 1)
{
    const size_t tab = size_t(d) * N * tab_entry_bytes(prec, kind);
    return ((tab + 127) & ~size_t(127)) + size_t(d) * N * 8 * size_t(rep);
}

// Device pointers of one problem's state.
struct ProblemPtrs {
    double* params;
    DevConst* cst;
    double* edges;
    double2* tab64;
    float* tab32;
    uint64_t* thr;
    double* partials;
    double* hslots;
    double* acc;
    double* last;
    double* records;
    int32_t* rec_flag;
    DevResult* result;
    double* adj_part;
};

inline ProblemPtrs problem_ptrs(void* ws, const Layout& L)
{
    char* b = static_cast<char*>(ws);
    ProblemPtrs p;
    p.params = reinterpret_cast<double*>(b + L.params);
    p.cst = reinterpret_cast<DevConst*>(b + L.cst);
    p.edges = reinterpret_cast<double*>(b + L.edges);
    p.tab64 = reinterpret_cast<double2*>(b + L.tab64);
    p.tab32 = reinterpret_cast<float*>(b + L.tab32);
    p.thr = reinterpret_cast<uint64_t*>(b + L.thr);
    p.partials = reinterpret_cast<double*>(b + L.partials);
    p.hslots = reinterpret_cast<double*>(b + L.hslots);
    p.acc = reinterpret_cast<double*>(b + L.acc);
    p.last = reinterpret_cast<double*>(b + L.last);
    p.records = reinterpret_cast<double*>(b + L.records);
    p.rec_flag = reinterpret_cast<int32_t*>(b + L.rec_flag);
    p.result = reinterpret_cast<DevResult*>(b + L.result);
    p.adj_part = reinterpret_cast<double*>(b + L.adj_part);
    return p;
}

// ---------------------------------------------------------------------------
// Kernel argument blocks.

struct SampleArgs {
    const DevConst* cst;
    const void* tab;     // double2* (FP64) or float2* (FP32), [d][N]
    const uint64_t* thr; // [d] Genz discontinuous thresholds
    double* partials;    // [gridDim.x][2]: S1, S2 (the histogram goes to hslots)
    double* hslots;      // [kHistSlots][d*N]: block b adds its histogram into slot (b / 8) mod kHistSlots
    uint64_t e0;         // first event index of this launch
    uint64_t n;          // events in this launch
    uint32_t t;          // iteration index
    uint32_t ctr3;       // problem index * 256
    uint32_t key0, key1; // seed
    int d, N;
    int hrep_log2;       // log2 of the histogram replicas per bin
    int hist;            // 0: no histograms this launch (only S1, S2 are written)
};

struct DumpArgs {
    const DevConst* cst;
    const void* tab;
    const uint64_t* thr;
    double* out;         // [n][3d+2]
    uint64_t e0, n;
    uint32_t t, ctr3, key0, key1;
    int d, N;
};

struct AdjointArgs {
    const DevConst* cst;
    const void* tab;
    double* partials;    // [gridDim.x][d+1]
    const double* gout;
    void* grad;          // [d+1], FP64 or (grad_fp32) FP32
    uint64_t n;
    uint32_t t, ctr3, key0, key1;
    int d, N;
    int grad_fp32;
};

enum MergeFlags {
    MERGE_BEGIN = 1,
    MERGE_END = 2,
    MERGE_NO_COMBINE = 4,
    MERGE_REFINE = 8,
    MERGE_NO_HIST = 16,
    MERGE_NO_RECORD = 32,  // statistics of the iteration kept as the last ones, not recorded
    MERGE_GRAD = 64        // one more block sums the gradient rows gpart into grad_out (times 1/M)
};

struct MergeArgs {
    const double* partials;  // [rows][rstride]: S1, S2 (and H when hslots is null)
    double* hslots;          // [kHistSlots][d*N] histogram accumulators, or null: the rows hold H
    double* acc;             // [2][pstride]
    double* last;            // [pstride]
    double* edges;           // [d][N+1]
    double2* tab64;
    float* tab32;
    uint64_t* thr;           // Genz discontinuous thresholds (rebuilt with the tables)
    const DevConst* cst;     // centres for the FP32 table
    double* records;
    int32_t* rec_flag;
    DevResult* result;
    double alpha;
    double M;                // events of the iteration (at END)
    const double* gpart;     // MERGE_GRAD: [rows][d + 1] gradient rows of the event kernel
    double* grad_out;        // MERGE_GRAD: [d + 1] (1/M) sum of the rows
    double* last_out;        // at END, when not null: (I_t, sigma_t) of the iteration
    int rows;
    int rstride;             // doubles per partial row: 2, or pstride when the rows hold H
    int d, N, pstride, kind;
    int flags;
    int rec_idx;
};

// ---------------------------------------------------------------------------
// Batches: many independent problems, each with its own grid.

// Device descriptor of one problem of a batch.
struct BatchProblem {
    const DevConst* cst;
    double* edges;
    double2* tab64;
    float* tab32;
    uint64_t* thr;
    double* last;       // S1, S2, H of the last iteration
    double* records;    // [n_iter][2]
    int32_t* rec_flag;
    DevResult* result;
    double alpha;
    double M;           // events per iteration
    uint32_t key0, key1, ctr3;
    int d, N, pstride;
    int first_item, n_items;
    uint64_t row0;      // first partial row (in doubles) of the problem's items
};

// One unit of work of the persistent event kernel: `n` events starting at
// event index e0 of problem `prob`; its partial row starts at row_off doubles.
struct BatchItem {
    int32_t prob;
    int32_t pad;
    uint64_t e0;
    uint64_t n;
    uint64_t row_off;
};

// Problems of a batch are grouped by dimension bucket (d <= 4, 8, 16, 32,
// 64); each bucket's items are contiguous and run in a launch of their own.
constexpr int kMaxBuckets = 5;

struct BatchArgs {
    const BatchProblem* probs;
    const BatchItem* items;
    double* partials;
    uint32_t* queue;    // this launch's work counter (the finish kernel re-arms all kMaxBuckets)
    int item_lo, item_hi;  // this launch takes items [item_lo, item_hi)
    int n_probs;
    uint32_t t;         // iteration index
    int hrep_log2;      // log2 of the histogram replicas per bin
};

#ifndef __HIPCC_RTC__
// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files).

hipError_t launch_sample(int prec, int kind, const SampleArgs& a, int blocks, int threads, hipStream_t s);
size_t sample_lds(int prec, int kind, int d, int N, int rep, bool hist = true);
hipError_t launch_dump(int prec, int kind, const DumpArgs& a, hipStream_t s);
hipError_t launch_sample_grad(int prec, const SampleArgs& a, double* gpart, int blocks, int threads, hipStream_t s);
hipError_t launch_grad_scale(const double* G, const double* gout, void* grad, int n, int grad_fp32, hipStream_t s);
hipError_t launch_adjoint(int prec, const AdjointArgs& a, int blocks, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_refine(const MergeArgs& a, hipStream_t s);   // from `last`, d blocks
hipError_t launch_prepare(int prec, int kind, int d, int N, const double* params, DevConst* cst,
                          hipStream_t s);
hipError_t launch_init_state(const ProblemPtrs& p, int d, int N, int pstride, hipStream_t s);
hipError_t launch_build_tables(const ProblemPtrs& p, int kind, int d, int N, hipStream_t s);
hipError_t launch_zero(double* x, size_t n, hipStream_t s);
hipError_t launch_combine(const double* records, const int32_t* rec_flag, int n_rec, DevResult* result,
                          hipStream_t s);
// rest: null (all n values in src), or values 1..n-1 (src holds value 0)
hipError_t launch_set_params(int prec, int kind, int d, int N, const void* src, int n, int is_fp32,
                             const ProblemPtrs& p, hipStream_t s, const void* rest = nullptr);
hipError_t launch_reset_results(double* records, int32_t* rec_flag, DevResult* result,
                                hipStream_t s);
hipError_t launch_copy_last(const DevResult* result, double* out2, hipStream_t s);
int sample_max_blocks_per_cu(int prec, int kind, int d, int N, int threads, int rep);

// Fixed histogram layout of the batch event kernel (buckets with d <= 16 whose
// problems all have n_bins <= kBatchFixBins, 8 or 16 replicas): fix_l2 = log2
// of the replicas, 0 for the general layout.
constexpr int kBatchFixBins = 64;
hipError_t launch_batch_sample(int prec, int kind, int dmax, size_t lds, const BatchArgs& a, int blocks,
                               int threads, bool hist, int fix_l2, hipStream_t s);
int batch_max_blocks_per_cu(int prec, int kind, int dmax, size_t lds, int threads, int fix_l2);
hipError_t launch_batch_finish(const BatchArgs& a, int dmax, int kind, int rec_idx, int flags, hipStream_t s);
hipError_t launch_batch_reset(const BatchArgs& a, int dmax, int n_rec, int kind, hipStream_t s);
hipError_t launch_batch_combine(const BatchArgs& a, int n_rec, hipStream_t s);
#endif

}  // namespace vegas
