// Event kernel of one Vegas iteration: points -> map -> integrand -> block
// partials of S1 = sum f w, S2 = sum (f w)^2 and H[i][b] = sum (f w)^2 over
// events in bin b of dimension i (the accumulators of Lepage's method that
// the paper's per-event stage fills, sec. 2.2).
//
// Layout: the grid's (lower edge, width) table [d][N] and the block's
// histogram [d][N] (FP64) live in LDS; events never touch memory.  Each
// thread strides over the launch's events; S1/S2 are Kahan-summed per thread,
// reduced across the block and written as the block's row (S1, S2) of the
// partial table (summed later in a fixed order); the block's histogram is
// added into one of kHistSlots accumulators with FP64 atomics (its sums come
// from LDS atomics in no fixed order anyway).
#include "device_common.hpp"

namespace vegas {

// Histogram modes of the event kernel:
//   kHistNone    no histograms (an iteration whose grid is not refined);
//   kHistGeneral table first, then the histogram with runtime strides;
//   kHistFixed   d in {4, 8, 12, 16}, N <= 64, 16 replicas: the histogram
//                starts the LDS block with a compile-time stride of 64 bins x
//                16 replicas (8 KiB) per dimension, so an atomic's address is
//                one shift-add of the bin onto the lane's replica offset and
//                the dimension's offset rides in the instruction's immediate
//                field; the grid table follows the histogram (at d = 16:
//                128 KiB + the table, one 1024-thread block per CU, as the
//                general layout's 16 replicas need anyway).
constexpr int kHistNone = 0, kHistGeneral = 1, kHistFixed = 2;
constexpr int kFixBins = 64;
constexpr int kFixRepLog2 = 4;
constexpr int kFixDimBytes = kFixBins << (kFixRepLog2 + 3);

// Fewest waves per SIMD the register allocation must allow.  6 (80 VGPRs) for
// the FP64 Gaussian, bimodal and product-peak kernels up to d = 8: they then
// fit without spills, and the launch runs two 768-thread blocks per CU (the
// fixed histogram layout's LDS admits two blocks), 6 waves per SIMD.  At 8
// waves (64 VGPRs, two 1024-thread blocks) the d = 8 Gaussian spilled 15
// registers and took 62.2-63.0 us per 1e7 events, at 7 (896-thread blocks)
// it still spilled 8 and took 70.0-70.8 us, at 6: 57.9-58.5 us.  4 elsewhere:
// the discontinuous integrand and larger d would spill heavily, and the
// FP32-mixed kernels reach 8 waves by themselves.
// The FP64 discontinuous integrand with histograms at d = 16: its 16 FP64
// c_i and thresholds leave too few scalar registers, and at 128 VGPRs (4
// waves) it spilled 18 of them (72 bytes per lane, 37.6 MB of scratch traffic
// per 1e7 events); it runs one 768-thread block per CU, 3 waves per SIMD,
// without spills: 132.1-132.3 -> 123.4-123.6 us per 1e7 events.  (At d = 13,
// in the guarded d <= 16 kernel, 3 waves ran slower: 167.0-167.6 -> 178.4-178.6.)
template <class P, int KIND, int DMAX, bool EXACT, int HM>
struct ThreeWaves {
    static constexpr bool value = P::is64 && KIND == GENZ_DISC && DMAX == 16 && EXACT && HM != 0;
};

template <class P, int KIND, int DMAX, bool EXACT = false, int HM = 0>
struct MinWaves {
    static constexpr int value =
        ThreeWaves<P, KIND, DMAX, EXACT, HM>::value ? 3 : (P::is64 && KIND != GENZ_DISC && DMAX <= 8) ? 6 : 4;
};

// Most waves per SIMD the kernel is compiled for.  Beyond d = 8 the kernels
// with histograms run one 1024-thread block per CU (their LDS holds one
// block's table and replicated histogram), i.e. 4 waves per SIMD, which the
// compiler cannot know from the dynamic LDS size: told so, it may use up to
// 128 registers and keep an event's table reads in flight together instead
// of waiting on each (the d = 20 bimodal kernel waited on every one).
template <class P, int KIND, int DMAX, bool EXACT, int HM>
struct MaxWaves {
    static constexpr int value = ThreeWaves<P, KIND, DMAX, EXACT, HM>::value ? 3 : (DMAX > 8 && HM != 0) ? 4 : 8;
};

template <class P, int KIND, int DMAX, bool EXACT, int HM>
struct MaxThreads {
    static constexpr int value = ThreeWaves<P, KIND, DMAX, EXACT, HM>::value ? 768 : kBlock;
};

template <class P, int KIND, int DMAX, bool EXACT, int HM>
__global__ __attribute__((amdgpu_flat_work_group_size(1, MaxThreads<P, KIND, DMAX, EXACT, HM>::value),
                          amdgpu_waves_per_eu(MinWaves<P, KIND, DMAX, EXACT, HM>::value,
                                              MaxWaves<P, KIND, DMAX, EXACT, HM>::value))) void k_sample(
    SampleArgs a)
{
    constexpr bool FIX = HM == kHistFixed;
    static_assert(!FIX || (EXACT && DMAX <= 16), "fixed layout: d <= 16 only");
    using tab_t = typename TabEntry<P, KIND>::type;
    extern __shared__ __align__(128) unsigned char smem[];
    const int dN = a.d * a.N;
    const size_t tab_bytes = (size_t(dN) * sizeof(tab_t) + 127) & ~size_t(127);
    // histogram [dim][bin][replica]: with 16 replicas every lane of a wave
    // adds into its own bank pair (lane mod 16), whatever its bin
    const int rl2 = FIX ? kFixRepLog2 : a.hrep_log2, rep = 1 << rl2;
    const int lrep = int(threadIdx.x) & (rep - 1);
    const size_t hist_bytes = HM == kHistNone ? 0
                              : FIX           ? size_t(DMAX) * kFixDimBytes
                                              : size_t(dN) * rep * sizeof(double);
    tab_t* tab = reinterpret_cast<tab_t*>(smem + (FIX ? hist_bytes : 0));
    double* hist = reinterpret_cast<double*>(smem + (FIX ? 0 : tab_bytes));
    double* red = reinterpret_cast<double*>(smem + tab_bytes + hist_bytes);
    // the lane's replica within the bin: byte offset lrep * 8 (fixed layout)
    unsigned char* hlane = smem + (lrep << 3);

    const tab_t* gtab = static_cast<const tab_t*>(a.tab);
    for (int k = threadIdx.x; k < dN; k += blockDim.x) tab[k] = gtab[k];
    {   // clear the histogram, 16 bytes per store (hist is 128-byte aligned), then an odd last double
        double2* h2 = reinterpret_cast<double2*>(hist);
        for (int k = threadIdx.x; k < int(hist_bytes / sizeof(double2)); k += blockDim.x)
            h2[k] = make_double2(0.0, 0.0);
        if ((hist_bytes & 8) && threadIdx.x == 0) hist[hist_bytes / sizeof(double) - 1] = 0.0;
    }
    __syncthreads();

    EvalConsts<P, KIND, DMAX> cst;
    cst.load(a.cst, a.thr, a.d);
    const int d = EXACT ? DMAX : a.d;
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    double g1 = 0.0, g2 = 0.0;
    int ng = 0;
    // event k = j * stride + threadIdx.x * gridDim.x + blockIdx.x in pass j:
    // the last, partial pass is spread over every block rather than a few
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t k = uint64_t(threadIdx.x) * gridDim.x + blockIdx.x; k < a.n; k += stride) {
        EventEval<P, KIND, DMAX, EXACT> ev;
        ev.run(cst, tab, a.e0 + k, a.t, a.ctr3, a.key0, a.key1, d, a.N);
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
        if constexpr (HM != kHistNone) {
#pragma unroll
            for (int i = 0; i < DMAX; ++i) {
                if (i < d) {
                    if constexpr (FIX)
                        lds_atomic_add(reinterpret_cast<double*>(hlane + (i * kFixDimBytes + (ev.b[i] << (kFixRepLog2 + 3)))), v2);
                    else
                        lds_atomic_add(&(hist + (i * a.N << rl2))[(ev.b[i] << rl2) | lrep], v2);
                }
            }
        }
    }
    kahan_add(s1, c1, g1);
    kahan_add(s2, c2, g2);

    // block_sum synchronises, which also completes every histogram atomic
    const double S1 = block_sum(s1 - c1, red);
    const double S2 = block_sum(s2 - c2, red);
    double* row = a.partials + size_t(blockIdx.x) * 2;
    if (threadIdx.x == 0) {
        row[0] = S1;
        row[1] = S2;
    }
    // the block's histogram (replicas summed) goes into slot
    // (blockIdx / 8) mod kHistSlots with device-scope FP64 atomics: no
    // histogram row to write and read back, and 8 slots keep the atomics on
    // one address few.  Workgroups go to the 8 XCDs round-robin, so each XCD's
    // blocks spread over all the slots (blockIdx mod 8 gave each XCD one slot
    // and ran about 1 % slower)
    double* slot = a.hslots + size_t((blockIdx.x >> 3) % kHistSlots) * dN;
    if constexpr (FIX) {
        // bin (i, b) of the fixed layout, 16 replicas read 2 at a time
        for (int k = threadIdx.x; k < DMAX * kFixBins; k += blockDim.x) {
            const int i = k / kFixBins, bb = k % kFixBins;
            if (bb < a.N) {
                const double2* h2 = reinterpret_cast<const double2*>(hist + (k << kFixRepLog2));
                double h = 0.0;
#pragma unroll
                for (int r = 0; r < (1 << kFixRepLog2) / 2; ++r) {
                    const double2 p = h2[r];
                    h += p.x;
                    h += p.y;
                }
                atomicAdd(&slot[i * a.N + bb], h);
            }
        }
    } else if constexpr (HM != kHistNone) {
        for (int k = threadIdx.x; k < dN; k += blockDim.x) {
            const int base = k << rl2;
            double h = 0.0;
            for (int r = 0; r < rep; ++r) h += hist[base + r];
            atomicAdd(&slot[k], h);
        }
    }
}

// Per-event records for parity checks: b, delta, x, w, f of each event.
template <class P, int KIND, int DMAX>
__global__ __launch_bounds__(kBlock) void k_dump(DumpArgs a)
{
    using tab_t = typename TabEntry<P, KIND>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int dN = a.d * a.N;
    tab_t* tab = reinterpret_cast<tab_t*>(smem);
    const tab_t* gtab = static_cast<const tab_t*>(a.tab);
    for (int k = threadIdx.x; k < dN; k += blockDim.x) tab[k] = gtab[k];
    __syncthreads();
    EvalConsts<P, KIND, DMAX> cst;
    cst.load(a.cst, a.thr, a.d);
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t k = uint64_t(blockIdx.x) * kBlock + threadIdx.x; k < a.n; k += stride) {
        EventEval<P, KIND, DMAX> ev;
        ev.run(cst, tab, a.e0 + k, a.t, a.ctr3, a.key0, a.key1, a.d, a.N);
        double* row = a.out + k * size_t(3 * a.d + 2);
        // x = centre + u; delta as the kernel represents it (FP32: (RN32(lo) +
        // h)/2^32, and u carries the factor S); w and f with their exponents
        const double ds = P::is64 ? 1.0 : double(cst.dscale);
#pragma unroll
        for (int i = 0; i < DMAX; ++i) {
            if (i < a.d) {
                row[i] = double(ev.b[i]);
                row[a.d + i] = P::is64 ? double(ev.del[i]) : double(ev.del[i]) * 0x1p-32 + cst.bc.h64;
                row[2 * a.d + i] = double(ev.u[i]) * ds + a.cst->cA64[i];
            }
        }
        row[3 * a.d] = ldexp(double(ev.wp), ev.ew) * cst.Cw;
        row[3 * a.d + 1] = ldexp(double(ev.F), ev.fe) * cst.Cf;
    }
}

// Adjoint at fixed samples (Gaussian): per-thread FP64 sums of
// v * d ln f / d theta_j, theta = (mu_0..mu_{d-1}, a):
//   d ln f / d mu_j = 2 (x_j - mu_j) / a^2,  d ln f / d a = (2 s / a^2 - d) / a.
// Block rows go to a partial table; k_adjoint_merge adds them in a fixed
// order and writes gout * sum / M.  EXACT: d == DMAX, so the per-dimension
// guards fold away and the table reads of an event can all be in flight.
template <class P, int DMAX, bool EXACT>
__global__ __launch_bounds__(kBlock) void k_adjoint(AdjointArgs a)
{
    using tab_t = typename TabEntry<P, GAUSS>::type;
    using real = typename P::real;
    extern __shared__ __align__(16) unsigned char smem[];
    const int dN = a.d * a.N;
    const size_t tab_bytes = (size_t(dN) * sizeof(tab_t) + 15) & ~size_t(15);
    tab_t* tab = reinterpret_cast<tab_t*>(smem);
    double* red = reinterpret_cast<double*>(smem + tab_bytes);
    const tab_t* gtab = static_cast<const tab_t*>(a.tab);
    for (int k = threadIdx.x; k < dN; k += blockDim.x) tab[k] = gtab[k];
    __syncthreads();

    const DevConst* c = a.cst;
    EvalConsts<P, GAUSS, DMAX> cst;
    cst.load(c, nullptr, a.d);
    // the FP32 path's u carries the factor S = 2^(ws + 32): its constants take S^-1, S^-2 (exact)
    const double ds = P::is64 ? 1.0 : double(c->dscale32) * 0x1p-32;
    const real ka = P::is64 ? real(c->kexp64) : real(double(c->ka32) * ds);
    // d ln f / d mu_j = 2 ka u_j: the events' sum of v u_j, then one product
    // with 2 ka per block row (the factor 2 is exact)
    const real ka2 = real(2) * ka;
    const double inv_a = c->inv_a;
    const int d = EXACT ? DMAX : a.d;
    const double ka64 = c->kexp64 * ds * ds;
    double g[DMAX + 1];
#pragma unroll
    for (int j = 0; j <= DMAX; ++j) g[j] = 0.0;

    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t k = uint64_t(blockIdx.x) * kBlock + threadIdx.x; k < a.n; k += stride) {
        EventEval<P, GAUSS, DMAX, EXACT> ev;
        ev.run(cst, tab, k, a.t, a.ctr3, a.key0, a.key1, d, a.N);
        const double v = ev.value(cst);
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
            if (j < d) g[j] += v * double(ev.u[j]);  // times 2 ka once per block
        const double da = 2.0 * ev.s64 * ka64 - double(d);
        g[DMAX] += v * (da * inv_a);
    }

    double* row = a.partials + size_t(blockIdx.x) * (d + 1);
#pragma unroll
    for (int j = 0; j <= DMAX; ++j) {
        if (j < d || j == DMAX) {
            const double t = block_sum(g[j], red);
            if (threadIdx.x == 0) row[j < d ? j : d] = j < d ? t * double(ka2) : t;
        }
    }
}

// Final step of the adjoint: the rows' fixed-order sums scaled by gout/M,
// stored in FP64 or rounded once to FP32 (grad_fp32).
__global__ __launch_bounds__(kMergeThreads) void k_adjoint_merge(AdjointArgs a, int rows)
{
    adjoint_merge_block(a.partials, rows, a.d, *a.gout / double(a.n), a.grad, a.grad_fp32);
}

// Forward pass with the gradient (Gaussian, frozen grid, no histograms):
// the event kernel without histograms -- same events per thread, same
// grouped Kahan S1, S2, so the estimate is bitwise that of k_sample -- that
// also sums each event's v d ln f / d theta_j, as k_adjoint does, into
// per-block rows gpart[block][d + 1] (merged by k_merge's gradient block).
// It launches like the event kernel (two 1024-thread blocks per CU, 8 waves
// per SIMD), so FP32 with d = 4 or 8 is compiled for 8 waves: at its natural
// 70 registers (d = 8) only one block fitted per CU and the grid ran in two
// rounds of 4 waves per SIMD.
template <class P, int DMAX, bool EXACT>
struct GradMinWaves {
    static constexpr int value = (!P::is64 && DMAX <= 8 && EXACT) ? 8 : 1;
};

template <class P, int DMAX, bool EXACT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GradMinWaves<P, DMAX, EXACT>::value))) void
k_sample_grad(SampleArgs a, double* gpart)
{
    using tab_t = typename TabEntry<P, GAUSS>::type;
    using real = typename P::real;
    extern __shared__ __align__(128) unsigned char smem[];
    const int dN = a.d * a.N;
    const size_t tab_bytes = (size_t(dN) * sizeof(tab_t) + 127) & ~size_t(127);
    tab_t* tab = reinterpret_cast<tab_t*>(smem);
    double* red = reinterpret_cast<double*>(smem + tab_bytes);
    const tab_t* gtab = static_cast<const tab_t*>(a.tab);
    for (int k = threadIdx.x; k < dN; k += blockDim.x) tab[k] = gtab[k];
    __syncthreads();

    const DevConst* c = a.cst;
    EvalConsts<P, GAUSS, DMAX> cst;
    cst.load(c, nullptr, a.d);
    const double ds = P::is64 ? 1.0 : double(c->dscale32) * 0x1p-32;
    const real ka = P::is64 ? real(c->kexp64) : real(double(c->ka32) * ds);
    const real ka2 = real(2) * ka;
    const double inv_a = c->inv_a;
    const int d = EXACT ? DMAX : a.d;
    const double ka64 = c->kexp64 * ds * ds;
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    double g1 = 0.0, g2 = 0.0;
    int ng = 0;
    double g[DMAX + 1];
#pragma unroll
    for (int j = 0; j <= DMAX; ++j) g[j] = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t k = uint64_t(threadIdx.x) * gridDim.x + blockIdx.x; k < a.n; k += stride) {
        EventEval<P, GAUSS, DMAX, EXACT> ev;
        ev.run(cst, tab, a.e0 + k, a.t, a.ctr3, a.key0, a.key1, d, a.N);
        double v, v2;
        {
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
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
            if (j < d) g[j] += v * double(ev.u[j]);  // times 2 ka once per block
        const double da = 2.0 * ev.s64 * ka64 - double(d);
        g[DMAX] += v * (da * inv_a);
    }
    kahan_add(s1, c1, g1);
    kahan_add(s2, c2, g2);
    const double S1 = block_sum(s1 - c1, red);
    const double S2 = block_sum(s2 - c2, red);
    if (threadIdx.x == 0) {
        double* row = a.partials + size_t(blockIdx.x) * 2;
        row[0] = S1;
        row[1] = S2;
    }
    double* grow = gpart + size_t(blockIdx.x) * (d + 1);
#pragma unroll
    for (int j = 0; j <= DMAX; ++j) {
        if (j < d || j == DMAX) {
            const double t = block_sum(g[j], red);
            if (threadIdx.x == 0) grow[j < d ? j : d] = j < d ? t * double(ka2) : t;
        }
    }
}

// ---------------------------------------------------------------------------
// Dispatch over (precision, integrand, dimension bucket).

static int dim_bucket(int d)
{
    if (d <= 4) return 4;
    if (d <= 8) return 8;
    if (d <= 12) return 12;
    if (d <= 16) return 16;
    if (d <= 20) return 20;
    if (d <= 24) return 24;
    if (d <= 32) return 32;
    if (d <= 48) return 48;
    return 64;
}

#define VEGAS_DMAX_SWITCH(DM, CALL)            \
    switch (DM) {                              \
    case 4: { constexpr int D_ = 4; CALL; }    \
    case 8: { constexpr int D_ = 8; CALL; }    \
    case 12: { constexpr int D_ = 12; CALL; }  \
    case 16: { constexpr int D_ = 16; CALL; }  \
    case 20: { constexpr int D_ = 20; CALL; }  \
    case 24: { constexpr int D_ = 24; CALL; }  \
    case 32: { constexpr int D_ = 32; CALL; }  \
    case 48: { constexpr int D_ = 48; CALL; }  \
    default: { constexpr int D_ = 64; CALL; }  \
    }

// The histogram mode of a launch: none, or the fixed layout where it applies
// (d in {4, 8, 12, 16}, N <= 64, 16 replicas), or the general one.
static int hist_mode(int d, int N, int rep, bool hist)
{
    if (!hist) return kHistNone;
    return (d == 4 || d == 8 || d == 12 || d == 16) && N <= kFixBins && rep == (1 << kFixRepLog2) ? kHistFixed
                                                                                                 : kHistGeneral;
}

template <class P, int KIND>
static const void* sample_fn(int d, int hm)
{
    if (hm == kHistFixed) {
        if (d == 4) return reinterpret_cast<const void*>(&k_sample<P, KIND, 4, true, kHistFixed>);
        if (d == 8) return reinterpret_cast<const void*>(&k_sample<P, KIND, 8, true, kHistFixed>);
        if (d == 12) return reinterpret_cast<const void*>(&k_sample<P, KIND, 12, true, kHistFixed>);
        return reinterpret_cast<const void*>(&k_sample<P, KIND, 16, true, kHistFixed>);
    }
    if (hm == kHistNone) {
        if (d == dim_bucket(d)) {
            VEGAS_DMAX_SWITCH(d, return reinterpret_cast<const void*>(&k_sample<P, KIND, D_, true, kHistNone>))
        }
        VEGAS_DMAX_SWITCH(dim_bucket(d), return reinterpret_cast<const void*>(&k_sample<P, KIND, D_, false, kHistNone>))
    }
    if (d == dim_bucket(d)) {
        VEGAS_DMAX_SWITCH(d, return reinterpret_cast<const void*>(&k_sample<P, KIND, D_, true, kHistGeneral>))
    }
    VEGAS_DMAX_SWITCH(dim_bucket(d), return reinterpret_cast<const void*>(&k_sample<P, KIND, D_, false, kHistGeneral>))
}

template <class P>
static const void* sample_fn_kind(int kind, int d, int hm)
{
    switch (kind) {
    case GAUSS: return sample_fn<P, GAUSS>(d, hm);
    case BIMODAL: return sample_fn<P, BIMODAL>(d, hm);
    case GENZ_DISC: return sample_fn<P, GENZ_DISC>(d, hm);
    default: return sample_fn<P, GENZ_PEAK>(d, hm);
    }
}

static const void* sample_kernel(int prec, int kind, int d, int N, int rep, bool hist)
{
    const int hm = hist_mode(d, N, rep, hist);
    return prec == FP64 ? sample_fn_kind<P64>(kind, d, hm) : sample_fn_kind<P32>(kind, d, hm);
}

template <class P, int KIND>
static const void* dump_fn(int d)
{
    VEGAS_DMAX_SWITCH(dim_bucket(d), return reinterpret_cast<const void*>(&k_dump<P, KIND, D_>))
}

template <class P>
static const void* dump_fn_kind(int kind, int d)
{
    switch (kind) {
    case GAUSS: return dump_fn<P, GAUSS>(d);
    case BIMODAL: return dump_fn<P, BIMODAL>(d);
    case GENZ_DISC: return dump_fn<P, GENZ_DISC>(d);
    default: return dump_fn<P, GENZ_PEAK>(d);
    }
}

template <class P>
static const void* adjoint_fn(int d)
{
    if (d == dim_bucket(d)) {
        VEGAS_DMAX_SWITCH(d, return reinterpret_cast<const void*>(&k_adjoint<P, D_, true>))
    }
    VEGAS_DMAX_SWITCH(dim_bucket(d), return reinterpret_cast<const void*>(&k_adjoint<P, D_, false>))
}

template <class P>
static const void* sample_grad_fn(int d)
{
    if (d == dim_bucket(d)) {
        VEGAS_DMAX_SWITCH(d, return reinterpret_cast<const void*>(&k_sample_grad<P, D_, true>))
    }
    VEGAS_DMAX_SWITCH(dim_bucket(d), return reinterpret_cast<const void*>(&k_sample_grad<P, D_, false>))
}

hipError_t launch_sample_grad(int prec, const SampleArgs& a, double* gpart, int blocks, int threads, hipStream_t s)
{
    const void* fn = prec == FP64 ? sample_grad_fn<P64>(a.d) : sample_grad_fn<P32>(a.d);
    const size_t tab = size_t(a.d) * a.N * tab_entry_bytes(prec, GAUSS);
    const size_t lds = ((tab + 127) & ~size_t(127)) + sizeof(double) * (kBlock / 64);
    void* args[] = {const_cast<SampleArgs*>(&a), &gpart};
    return hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, lds, s);
}

size_t sample_lds(int prec, int kind, int d, int N, int rep, bool hist)
{
    // the wave partials of the block sums follow the table and histogram
    const size_t red = sizeof(double) * (kBlock / 64);
    switch (hist_mode(d, N, rep, hist)) {
    case kHistNone: return lds_bytes(prec, kind, d, N, 0) + red;
    case kHistFixed: return size_t(d) * kFixDimBytes + lds_bytes(prec, kind, d, N, 0) + red;
    default: return lds_bytes(prec, kind, d, N, rep) + red;
    }
}

hipError_t launch_sample(int prec, int kind, const SampleArgs& a, int blocks, int threads, hipStream_t s)
{
    const int rep = 1 << a.hrep_log2;
    const bool hist = a.hist != 0;
    const void* fn = sample_kernel(prec, kind, a.d, a.N, rep, hist);
    void* args[] = {const_cast<SampleArgs*>(&a)};
    return hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, sample_lds(prec, kind, a.d, a.N, rep, hist), s);
}

hipError_t launch_dump(int prec, int kind, const DumpArgs& a, hipStream_t s)
{
    const void* fn = prec == FP64 ? dump_fn_kind<P64>(kind, a.d) : dump_fn_kind<P32>(kind, a.d);
    const size_t tab = size_t(a.d) * a.N * tab_entry_bytes(prec, kind);
    const size_t lds = tab;
    uint64_t blocks = (a.n + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    void* args[] = {const_cast<DumpArgs*>(&a)};
    return hipLaunchKernel(fn, dim3(unsigned(blocks)), dim3(kBlock), args, lds, s);
}

hipError_t launch_adjoint(int prec, const AdjointArgs& a, int blocks, hipStream_t s)
{
    const void* fn = prec == FP64 ? adjoint_fn<P64>(a.d) : adjoint_fn<P32>(a.d);
    const size_t tab = size_t(a.d) * a.N * tab_entry_bytes(prec, GAUSS);
    const size_t lds = ((tab + 15) & ~size_t(15)) + sizeof(double) * (kBlock / 64);
    void* args[] = {const_cast<AdjointArgs*>(&a)};
    hipError_t e = hipLaunchKernel(fn, dim3(blocks), dim3(kBlock), args, lds, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adjoint_merge, dim3(1), dim3(kMergeThreads), 0, s, a, blocks);
    return hipGetLastError();
}

int sample_max_blocks_per_cu(int prec, int kind, int d, int N, int threads, int rep)
{
    int n = 0;
    const void* fn = sample_kernel(prec, kind, d, N, rep, true);
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, fn) == hipSuccess && threads > at.maxThreadsPerBlock) return 0;  // not launchable
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, sample_lds(prec, kind, d, N, rep, true)) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace vegas
