// Batched Vegas iterations: many independent problems (own dimension, grid,
// event count and integrand parameters) in one persistent launch.
//
// The event kernel's blocks take work items -- a tile of events of one
// problem -- from an atomic counter until none is left.  Items are ordered by
// cost (larger dimension first), so the tail of the launch is made of cheap
// items.  When a block moves to another problem it reloads that problem's
// grid table into LDS; each item leaves one partial row (S1, S2, H[d][N]).
// The finish kernel then reduces each problem's rows (one block per problem
// and column group), records the iteration and refines the grid, as the
// single-problem reduction does.
#include "grid_ops.hpp"

namespace vegas {

// Fewest waves per SIMD the register allocation must allow: 4, i.e. up to
// 128 registers.  The FP32-mixed kernel of the d <= 16 bucket needs about
// 100; capped at 80 (6 waves) it spilled 30 registers to scratch, which
// moved about 9 GB per launch through HBM for the 256-problem batch (its
// histogram launches took 22 ms per run against 18 ms without the spills).
template <class P, int DMAX>
struct BatchMinWaves {
    static constexpr int value = 4;
};

// The events of one work item into the block's LDS histogram and the item's
// (S1, S2) row.  DE > 0: compiled for exactly DE dimensions (the problem's
// d), with no per-dimension guards, so the whole event runs as one block of
// straight-line code; DE = 0: each dimension is guarded against d <= DMAX.
// hist/hlane: the general layout's histogram, or the fixed layout's lane
// base (FRL2 > 0).
template <class P, int KIND, int DMAX, int DE, bool HIST, int FRL2>
__device__ __forceinline__ void batch_item_events(const BatchArgs& a, const BatchItem& it, const BatchProblem& pr,
                                                  const typename TabEntry<P, KIND>::type* tab, double* hist,
                                                  unsigned char* hlane, int rl2, int lrep, int d, int N, double* red)
{
    constexpr bool FIX = HIST && FRL2 > 0;
    constexpr int kDimBytes = kBatchFixBins << (FRL2 + 3);
    constexpr int DM = DE > 0 ? DE : DMAX;
    EvalConsts<P, KIND, DM> cst;
    cst.load(pr.cst, pr.thr, d);
    const uint32_t key0 = pr.key0, key1 = pr.key1, ctr3 = pr.ctr3;
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0, g1 = 0.0, g2 = 0.0;
    int ng = 0;
    for (uint64_t k = threadIdx.x; k < it.n; k += blockDim.x) {
        EventEval<P, KIND, DM, (DE > 0)> ev;
        ev.run(cst, tab, it.e0 + k, a.t, ctr3, key0, key1, d, N);
        double v, v2;
        {
            // rounded as written in every variant (with or without histograms)
#pragma clang fp contract(off)
            v = ev.value(cst);
            v2 = v * v;
            g1 += v;
            g2 += v2;
        }
        if (++ng == kGroup) {
            kahan_add(s1, c1, g1);
            kahan_add(s2, c2, g2);
            g1 = g2 = 0.0;
            ng = 0;
        }
        if constexpr (FIX) {
#pragma unroll
            for (int i = 0; i < DM; ++i)
                if (DE > 0 || i < d)
                    lds_atomic_add(reinterpret_cast<double*>(hlane + (i * kDimBytes + (ev.b[i] << (FRL2 + 3)))), v2);
        } else if constexpr (HIST) {
#pragma unroll
            for (int i = 0; i < DM; ++i)
                if (DE > 0 || i < d) lds_atomic_add(&(hist + (i * N << rl2))[(ev.b[i] << rl2) | lrep], v2);
        }
    }
    (void)lrep;
    kahan_add(s1, c1, g1);
    kahan_add(s2, c2, g2);
    // block_sum synchronises, which also completes every histogram atomic
    const double S1 = block_sum(s1 - c1, red);
    const double S2 = block_sum(s2 - c2, red);
    double* row = a.partials + it.row_off;
    if (threadIdx.x == 0) {
        row[0] = S1;
        row[1] = S2;
    }
}

// The exact-d variant for d in [LO, DE] (an if-chain from DE down), the
// guarded one below LO.
template <class P, int KIND, int DMAX, int DE, int LO, bool HIST, int FRL2>
__device__ __forceinline__ void batch_item_dispatch(const BatchArgs& a, const BatchItem& it, const BatchProblem& pr,
                                                    const typename TabEntry<P, KIND>::type* tab, double* hist,
                                                    unsigned char* hlane, int rl2, int lrep, int d, int N, double* red)
{
    if constexpr (DE < LO) {
        batch_item_events<P, KIND, DMAX, 0, HIST, FRL2>(a, it, pr, tab, hist, hlane, rl2, lrep, d, N, red);
    } else {
        if (d == DE)
            batch_item_events<P, KIND, DMAX, DE, HIST, FRL2>(a, it, pr, tab, hist, hlane, rl2, lrep, d, N, red);
        else
            batch_item_dispatch<P, KIND, DMAX, DE - 1, LO, HIST, FRL2>(a, it, pr, tab, hist, hlane, rl2, lrep, d, N,
                                                                       red);
    }
}

// Fixed histogram layout (FRL2 = log2 of the replicas, 3 or 4; 0: general),
// for buckets whose problems all have N <= kBatchFixBins: the histogram
// starts the LDS with a compile-time stride of 64 bins x 2^FRL2 replicas per
// dimension, so an atomic's address is one shift-add of the bin onto the
// lane's replica offset, with the dimension's offset in the instruction's
// immediate field; the problem's grid table follows it.
// The Gaussian's buckets up to d = 16 run each item with the loop compiled
// for the problem's exact d (items are sorted by d, so a block seldom
// changes variant); other integrands and larger buckets guard each dimension.
template <class P, int KIND, int DMAX, bool HIST, int FRL2>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(BatchMinWaves<P, DMAX>::value, 8))) void k_batch_sample(
    BatchArgs a)
{
    constexpr bool FIX = HIST && FRL2 > 0;
    static_assert(!FIX || DMAX <= 16, "fixed layout: d <= 16 only");
    constexpr int kDimBytes = kBatchFixBins << (FRL2 + 3);
    constexpr size_t kFixBytes = FIX ? size_t(DMAX) * kDimBytes : 0;
    // the bucket's d range: (DMAX/2, DMAX], and 1..4 for the smallest
    constexpr int kLo = DMAX <= 4 ? 1 : DMAX / 2 + 1;
    constexpr bool kExact = KIND == GAUSS && DMAX <= 16;
    using tab_t = typename TabEntry<P, KIND>::type;
    extern __shared__ __align__(128) unsigned char smem[];
    __shared__ int s_item;
    __shared__ double red[kBlock / 64];
    // histogram [dim][bin][replica], lane l adding into replica l mod rep
    const int rl2 = FIX ? FRL2 : a.hrep_log2, rep = 1 << rl2;
    const int lrep = int(threadIdx.x) & (rep - 1);
    int cur = -1;
    int d = 0, N = 0, dN = 0;
    tab_t* tab = reinterpret_cast<tab_t*>(smem + kFixBytes);
    double* hist = FIX ? reinterpret_cast<double*>(smem) : nullptr;
    // the lane's replica within the bin: byte offset lrep * 8 (fixed layout)
    unsigned char* hlane = smem + (lrep << 3);
    for (;;) {
        if (threadIdx.x == 0) s_item = a.item_lo + int(atomicAdd(a.queue, 1u));
        __syncthreads();
        const int item = s_item;
        if (item >= a.item_hi) break;  // every block leaves once the queue is empty
        const BatchItem it = a.items[item];
        const BatchProblem& pr = a.probs[it.prob];
        if (it.prob != cur) {
            cur = it.prob;
            d = pr.d;
            N = pr.N;
            dN = d * N;
            const tab_t* gtab = P::is64 ? reinterpret_cast<const tab_t*>(pr.tab64)
                                        : reinterpret_cast<const tab_t*>(pr.tab32);
            for (int k = threadIdx.x; k < dN; k += blockDim.x) tab[k] = gtab[k];
            if constexpr (!FIX) hist = reinterpret_cast<double*>(smem + ((size_t(dN) * sizeof(tab_t) + 127) & ~size_t(127)));
        }
        if constexpr (HIST) {
            const int nh = (FIX ? d * kBatchFixBins : dN) << rl2;
            for (int k = threadIdx.x; k < nh; k += blockDim.x) hist[k] = 0.0;
        }
        __syncthreads();

        if constexpr (kExact)
            batch_item_dispatch<P, KIND, DMAX, DMAX, kLo, HIST, FRL2>(a, it, pr, tab, hist, hlane, rl2, lrep, d, N,
                                                                     red);
        else
            batch_item_events<P, KIND, DMAX, 0, HIST, FRL2>(a, it, pr, tab, hist, hlane, rl2, lrep, d, N, red);

        if constexpr (HIST) {
            double* row = a.partials + it.row_off;
            for (int k = threadIdx.x; k < dN; k += blockDim.x) {
                // bin (i, b) of the row at k = i N + b; fixed layout: 64 bins per dimension
                const int hk = FIX ? k + (k / N) * (kBatchFixBins - N) : k;
                double h = 0.0;
                for (int r = 0; r < rep; ++r) h += hist[(hk << rl2) + r];
                row[2 + k] = h;
            }
        }
        __syncthreads();
    }
}

// Per problem and column group: reduce the problem's item rows, record the
// iteration, refine (adaptation iterations).  Also resets the work queue for
// the next event launch on the stream.
__global__ __launch_bounds__(kMergeThreads) void k_batch_finish(BatchArgs a, int kind, int rec_idx, int flags)
{
    const int g = blockIdx.x, p = blockIdx.y;
    if (p == 0 && g == 0 && threadIdx.x < kMaxBuckets) a.queue[threadIdx.x] = 0u;
    const BatchProblem pr = a.probs[p];
    if (g > pr.d) return;
    MergeArgs m{};
    m.partials = a.partials + pr.row0;
    m.acc = nullptr;
    m.last = pr.last;
    m.edges = pr.edges;
    m.tab64 = pr.tab64;
    m.tab32 = pr.tab32;
    m.thr = pr.thr;
    m.cst = pr.cst;
    m.records = pr.records;
    m.rec_flag = pr.rec_flag;
    m.result = pr.result;
    m.alpha = pr.alpha;
    m.M = pr.M;
    m.rows = pr.n_items;
    m.d = pr.d;
    m.N = pr.N;
    m.pstride = pr.pstride;
    m.rstride = pr.pstride;  // batch rows carry S1, S2 and H
    m.kind = kind;
    m.flags = MERGE_BEGIN | MERGE_END | flags;
    m.rec_idx = rec_idx;
    merge_group(m, g);
}

// Restart every problem: uniform grid and tables, no recorded iterations.
__global__ __launch_bounds__(kMergeThreads) void k_batch_reset(BatchArgs a, int n_rec, int kind)
{
    const int g = blockIdx.x, p = blockIdx.y;
    if (p == 0 && g == 0 && threadIdx.x < kMaxBuckets) a.queue[threadIdx.x] = 0u;
    const BatchProblem pr = a.probs[p];
    if (g < pr.d) {
        double* E = pr.edges + size_t(g) * (pr.N + 1);
        for (int k = threadIdx.x; k <= pr.N; k += blockDim.x) E[k] = double(k) / double(pr.N);
        __syncthreads();
        write_tables(g, E, pr.cst, kind, pr.N, pr.tab64, pr.tab32, pr.thr);
    } else if (g == pr.d) {
        for (int k = threadIdx.x; k < pr.pstride; k += blockDim.x) pr.last[k] = 0.0;
        for (int k = threadIdx.x; k < 2 * n_rec; k += blockDim.x) pr.records[k] = 0.0;
        for (int k = threadIdx.x; k < n_rec; k += blockDim.x) pr.rec_flag[k] = 0;
        if (threadIdx.x == 0) {
            const double nan = __builtin_nan("");
            DevResult* R = pr.result;
            R->integral = R->sigma = R->chi2_dof = R->last_integral = R->last_var = nan;
            R->n_iter = R->n_combined = R->n_events = R->n_nonfinite = 0;
        }
    }
}

__global__ void k_batch_combine(BatchArgs a, int n_rec)
{
    if (threadIdx.x != 0) return;
    const BatchProblem pr = a.probs[blockIdx.x];
    const int n = pr.result->n_iter < n_rec ? int(pr.result->n_iter) : n_rec;
    combine_records(pr.records, pr.rec_flag, n, pr.result);
}

hipError_t launch_batch_combine(const BatchArgs& a, int n_rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_combine, dim3(a.n_probs), dim3(64), 0, s, a, n_rec);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchArgs& a, int dmax, int kind, int rec_idx, int flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_finish, dim3(dmax + 1, a.n_probs), dim3(kMergeThreads), 0, s, a, kind, rec_idx, flags);
    return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchArgs& a, int dmax, int n_rec, int kind, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(dmax + 1, a.n_probs), dim3(kMergeThreads), 0, s, a, n_rec, kind);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

template <class P, int KIND, bool HIST>
static const void* batch_fn(int dmax, int fix_l2)
{
    if constexpr (HIST) {
        if (fix_l2 == 3 || fix_l2 == 4) {
            const bool r16 = fix_l2 == 4;
            switch (dmax) {
            case 4: return r16 ? reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 4, true, 4>)
                               : reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 4, true, 3>);
            case 8: return r16 ? reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 8, true, 4>)
                               : reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 8, true, 3>);
            case 16: return r16 ? reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 16, true, 4>)
                                : reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 16, true, 3>);
            default: break;
            }
        }
    }
    switch (dmax) {
    case 4: return reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 4, HIST, 0>);
    case 8: return reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 8, HIST, 0>);
    case 16: return reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 16, HIST, 0>);
    case 32: return reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 32, HIST, 0>);
    default: return reinterpret_cast<const void*>(&k_batch_sample<P, KIND, 64, HIST, 0>);
    }
}

template <class P, bool HIST>
static const void* batch_fn_kind(int kind, int dmax, int fix_l2)
{
    switch (kind) {
    case GAUSS: return batch_fn<P, GAUSS, HIST>(dmax, fix_l2);
    case BIMODAL: return batch_fn<P, BIMODAL, HIST>(dmax, fix_l2);
    case GENZ_DISC: return batch_fn<P, GENZ_DISC, HIST>(dmax, fix_l2);
    default: return batch_fn<P, GENZ_PEAK, HIST>(dmax, fix_l2);
    }
}

static const void* batch_kernel(int prec, int kind, int dmax, bool hist, int fix_l2)
{
    if (hist)
        return prec == FP64 ? batch_fn_kind<P64, true>(kind, dmax, fix_l2) : batch_fn_kind<P32, true>(kind, dmax, fix_l2);
    return prec == FP64 ? batch_fn_kind<P64, false>(kind, dmax, 0) : batch_fn_kind<P32, false>(kind, dmax, 0);
}

// Without histograms the launch keeps the same grid (and LDS size): it is a
// work queue, so residency only sets how many blocks share the items.
hipError_t launch_batch_sample(int prec, int kind, int dmax, size_t lds, const BatchArgs& a, int blocks,
                               int threads, bool hist, int fix_l2, hipStream_t s)
{
    void* args[] = {const_cast<BatchArgs*>(&a)};
    return hipLaunchKernel(batch_kernel(prec, kind, dmax, hist, fix_l2), dim3(blocks), dim3(threads), args, lds, s);
}

int batch_max_blocks_per_cu(int prec, int kind, int dmax, size_t lds, int threads, int fix_l2)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel(prec, kind, dmax, true, fix_l2), threads, lds) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace vegas
