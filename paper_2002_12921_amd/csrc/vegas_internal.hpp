// Internal declarations shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace vegas {

constexpr int kMaxDim = 64;
constexpr int kMaxBins = 255;
constexpr int kMaxParams = 1 + 2 * kMaxDim;
constexpr int kMaxRecords = 1024;   // recorded iterations per context
constexpr int kBlock = 256;         // threads per block of the event kernels
constexpr int kMaxBlocks = 4096;    // rows of the per-block partial table
constexpr int kMaxSplits = 64;      // row splits of the merge (level-2 rows)
constexpr size_t kLdsLimit = 160 * 1024;

enum Kind { GAUSS = 0, BIMODAL = 1, GENZ_DISC = 2, GENZ_PEAK = 3 };
enum Prec { FP64 = 0, FP32 = 1 };

// Derived per-problem constants, computed on the device from the raw FP64
// parameters whenever they change.  The event kernels compute
//   F  = unnormalised integrand in the kernel precision (at most ~1),
//   wp = product of the bin widths (FP32: times 2^wshift per dimension),
// and the event value v = f w = (double)(F * wp) * C with C = Cf * Cw,
// Cf the integrand normalisation and Cw = N^d (FP32: N^d 2^(-wshift d)).
struct DevConst {
    double C;        // Cf * Cw
    double Cf;       // f = Cf * F
    double Cw;       // w = wp * Cw
    double kexp64;   // Gaussian forms: 1/a^2
    double inv_a;    // Gaussian forms: 1/a (adjoint)
    double nscale;   // N / 2^32   (binning: yN = k * nscale + nhalf, exact)
    double nhalf;    // N / 2^33
    float kexp32;    // Gaussian forms: log2(e)/a^2
    float wgroup32;  // 2^(4 wshift): FP32 rescale after each full group of 4 dims
    float wlast32;   // 2^((d mod 4) wshift): after a final partial group
    float ka32;      // Gaussian forms: RN32(1/a^2) (adjoint)
    double p1_64[kMaxDim];  // GAUSS mu | BIMODAL muA | DISC c | PEAK c^2
    double p2_64[kMaxDim];  //          | BIMODAL muB | DISC a | PEAK a
    float p1_32[kMaxDim];   // FP32 forms (DISC: c log2(e))
    float p2_32[kMaxDim];
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
    size_t tab32;     // float2[d][N]   (RN32 of each)
    size_t partials;  // double[kMaxBlocks][pstride]
    size_t level2;    // double[kMaxSplits][pstride]
    size_t acc;       // double[2][pstride]   chunk accumulators (hi, lo)
    size_t last;      // double[pstride]      S1, S2, H of the last completed iteration
    size_t records;   // double[kMaxRecords][2]  (I_t, var_t)
    size_t rec_flag;  // int32[kMaxRecords]      combined?
    size_t result;    // DevResult
    size_t tickets;   // uint32[kMaxDim + 8]
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
    L.tab32 = take(sizeof(float) * 2 * d * N);
    L.partials = take(sizeof(double) * size_t(kMaxBlocks) * ps);
    L.level2 = take(sizeof(double) * size_t(kMaxSplits) * ps);
    L.acc = take(sizeof(double) * 2 * size_t(ps));
    L.last = take(sizeof(double) * size_t(ps));
    L.records = take(sizeof(double) * 2 * kMaxRecords);
    L.rec_flag = take(sizeof(int32_t) * kMaxRecords);
    L.result = take(sizeof(DevResult));
    L.tickets = take(sizeof(uint32_t) * (kMaxDim + 8));
    L.adj_part = take(sizeof(double) * size_t(kMaxBlocks) * (kMaxDim + 1));
    L.total = o;
    L.pstride = ps;
    return L;
}

inline size_t lds_bytes(int prec, int d, int N)
{
    const size_t tab = size_t(d) * N * (prec == FP64 ? 16 : 8);
    return ((tab + 15) & ~size_t(15)) + size_t(d) * N * 8;
}

// Device pointers of one problem's state.
struct ProblemPtrs {
    double* params;
    DevConst* cst;
    double* edges;
    double2* tab64;
    float2* tab32;
    double* partials;
    double* level2;
    double* acc;
    double* last;
    double* records;
    int32_t* rec_flag;
    DevResult* result;
    uint32_t* tickets;
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
    p.tab32 = reinterpret_cast<float2*>(b + L.tab32);
    p.partials = reinterpret_cast<double*>(b + L.partials);
    p.level2 = reinterpret_cast<double*>(b + L.level2);
    p.acc = reinterpret_cast<double*>(b + L.acc);
    p.last = reinterpret_cast<double*>(b + L.last);
    p.records = reinterpret_cast<double*>(b + L.records);
    p.rec_flag = reinterpret_cast<int32_t*>(b + L.rec_flag);
    p.result = reinterpret_cast<DevResult*>(b + L.result);
    p.tickets = reinterpret_cast<uint32_t*>(b + L.tickets);
    p.adj_part = reinterpret_cast<double*>(b + L.adj_part);
    return p;
}

// ---------------------------------------------------------------------------
// Kernel argument blocks.

struct SampleArgs {
    const DevConst* cst;
    const void* tab;     // double2* (FP64) or float2* (FP32), [d][N]
    double* partials;    // [gridDim.x][pstride]: S1, S2, H[d][N]
    uint64_t e0;         // first event index of this launch
    uint64_t n;          // events in this launch
    uint32_t t;          // iteration index
    uint32_t ctr3;       // problem index * 256
    uint32_t key0, key1; // seed
    int d, N, pstride;
};

struct DumpArgs {
    const DevConst* cst;
    const void* tab;
    double* out;         // [n][3d+2]
    uint64_t e0, n;
    uint32_t t, ctr3, key0, key1;
    int d, N;
};

struct AdjointArgs {
    const DevConst* cst;
    const void* tab;
    double* partials;    // [gridDim.x][d+1]
    uint32_t* ticket;
    const double* gout;
    double* grad;        // [d+1]
    uint64_t n;
    uint32_t t, ctr3, key0, key1;
    int d, N;
};

enum MergeFlags { MERGE_BEGIN = 1, MERGE_END = 2, MERGE_NO_COMBINE = 4, MERGE_REFINE = 8 };

struct MergeArgs {
    const double* partials;  // [rows][pstride]
    double* level2;          // [splits][pstride]
    double* acc;             // [2][pstride]
    double* last;            // [pstride]
    uint32_t* tickets;       // [d+1]
    double* edges;           // [d][N+1]
    double2* tab64;
    float2* tab32;
    double* records;
    int32_t* rec_flag;
    DevResult* result;
    double alpha;
    double M;                // events of the iteration (at END)
    int rows, splits;
    int d, N, pstride;
    int flags;
    int rec_idx;
};

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files).

hipError_t launch_sample(int prec, int kind, const SampleArgs& a, int blocks, hipStream_t s);
hipError_t launch_dump(int prec, int kind, const DumpArgs& a, hipStream_t s);
hipError_t launch_adjoint(int prec, const AdjointArgs& a, int blocks, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_refine(const MergeArgs& a, hipStream_t s);   // from `last`, d blocks
hipError_t launch_prepare(int prec, int kind, int d, int N, const double* params, DevConst* cst,
                          hipStream_t s);
hipError_t launch_init_state(const ProblemPtrs& p, int d, int N, int pstride, hipStream_t s);
hipError_t launch_build_tables(double* edges, double2* tab64, float2* tab32, int d, int N,
                               hipStream_t s);
hipError_t launch_params_from(const void* src, int n, int is_fp32, double* dst, hipStream_t s);
hipError_t launch_reset_results(double* records, int32_t* rec_flag, DevResult* result,
                                hipStream_t s);
hipError_t launch_copy_last(const DevResult* result, double* out2, hipStream_t s);
int sample_max_blocks_per_cu(int prec, int kind, int d, int N);

}  // namespace vegas
