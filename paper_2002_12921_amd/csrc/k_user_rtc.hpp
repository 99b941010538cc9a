// Event and dump kernels for an integrand compiled at run time from the
// caller's source (the paper's route for integrands written in C, C++ or GPU
// code and linked into the integrator, sec. 2.3).  This header is not built
// with the library: the host hands it, with vegas_internal.hpp and
// device_common.hpp, to the runtime compiler once per context, after the
// caller's source, with
//   VEGAS_DIM      the dimension d (a compile-time constant, so the point
//                  stays in registers and the caller's loops unroll),
//   VEGAS_THREADS  the largest block the event kernel is launched with,
//   VEGAS_FP32     defined for an FP32-mixed context,
// and vegas_real typedef'd to float (FP32-mixed) or double (FP64).  The
// caller's source defines
//   __device__ vegas_real vegas_integrand(const vegas_real* x, int dim, const double* params)
// evaluated at the mapped point x[0..d-1] in [0,1)^d; params is the context's
// parameter array in device memory.
//
// Everything but the integrand is the built-in event kernel's path in the
// context's precision: the same Philox words, exact bins, map and Jacobian
// N^d prod W_b, the same grouped-Kahan FP64 sums of v = f w and v^2, and the
// same per-dimension, per-bin FP64 histograms of v^2 (LDS replicas, then the
// block's histogram added into slot (blockIdx / 8) mod kHistSlots), so the
// reduction, refinement and combination kernels of the library serve it
// unchanged.
#pragma once

#include "device_common.hpp"

namespace vegas {
namespace user {

constexpr int D = VEGAS_DIM;
static_assert(D >= 1 && D <= kMaxDim, "VEGAS_DIM out of range");

__device__ __forceinline__ BinConsts bin_consts(int N, const DevConst* c)
{
    BinConsts bc;
    bc.mul = uint32_t(N);
    bc.add = uint32_t(N) >> 1;
    bc.h64 = (N & 1) ? 0x1p-33 : 0.0;
    bc.s32 = c->two_m32;
    return bc;
}

#ifdef VEGAS_FP32
// FP32-mixed context.  The table is the built-in FP32 one with centre 0:
// entry (RN32((E_b + h W / 2^32) S), RN32(W) 2^ws), S = 2^(ws + 32), so
// x S = fma(RN32(lo), W 2^ws, first entry) in FP32 and x = (x S) / S exactly;
// the width product is kept in FP32 with its binary exponent moved out every
// 8 dimensions, and the value f w = 2^ew (f wp) C is formed in FP64.
using tab_t = float2;
struct Event {
    int b[D];
    float del[D];  // RN32(lo)
    float x[D];
    float wp;
    int ew;

    __device__ __forceinline__ void run(const tab_t* __restrict__ tab, const BinConsts& bc, uint64_t e, uint32_t t,
                                        uint32_t ctr3, uint32_t key0, uint32_t key1, int N, float ds)
    {
#pragma clang fp contract(off)
        const uint32_t elo = uint32_t(e), ehi = uint32_t(e >> 32);
        float w = 1.0f;
        int ewl = 0;
#pragma unroll
        for (int g = 0; g < (D + 3) / 4; ++g) {
            const U4 k = philox4x32_10(elo, ehi, t, ctr3 + uint32_t(g), key0, key1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * g + q;
                if (i < D) {
                    int bi;
                    uint32_t lo;
                    bin_words(k.w[q], bc, bi, lo);
                    const tab_t tb = (tab + i * N)[bi];
                    const float dl = float(lo);
                    b[i] = bi;
                    del[i] = dl;
                    x[i] = fmaf(dl, tb.y, tb.x) * ds;
                    w *= tb.y;
                }
            }
            if ((g & 1) == 1 && 4 * g + 4 < D) {
                int e2;
                w = frexpf(w, &e2);
                ewl += e2;
            }
        }
        wp = w;
        ew = ewl;
    }
    __device__ __forceinline__ double delta(int i, const BinConsts& bc) const { return double(del[i]) * 0x1p-32 + bc.h64; }
    __device__ __forceinline__ double weight(double Cw) const { return ldexp(double(wp), ew) * Cw; }
    __device__ __forceinline__ double value(float f, double C) const
    {
#pragma clang fp contract(off)
        return ldexp(double(f) * double(wp), ew) * C;  // the product of two floats is exact in FP64
    }
};
#else
// FP64 context: delta = (lo + h)/2^32 is exact, x_i = fma(delta, W_b, E_b),
// the built-in FP64 map with centre 0 (the table of a user context holds E_b
// itself).
using tab_t = double2;
struct Event {
    int b[D];
    double del[D];
    double x[D];
    double wp;

    __device__ __forceinline__ void run(const tab_t* __restrict__ tab, const BinConsts& bc, uint64_t e, uint32_t t,
                                        uint32_t ctr3, uint32_t key0, uint32_t key1, int N, float)
    {
#pragma clang fp contract(off)
        const uint32_t elo = uint32_t(e), ehi = uint32_t(e >> 32);
        double w = 1.0;
#pragma unroll
        for (int g = 0; g < (D + 3) / 4; ++g) {
            const U4 k = philox4x32_10(elo, ehi, t, ctr3 + uint32_t(g), key0, key1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * g + q;
                if (i < D) {
                    int bi;
                    uint32_t lo;
                    bin_words(k.w[q], bc, bi, lo);
                    const tab_t tb = (tab + i * N)[bi];
                    const double dl = fma(double(lo), bc.s32, bc.h64);
                    b[i] = bi;
                    del[i] = dl;
                    x[i] = fma(dl, tb.y, tb.x);
                    w *= tb.y;
                }
            }
        }
        wp = w;
    }
    __device__ __forceinline__ double delta(int i, const BinConsts&) const { return del[i]; }
    __device__ __forceinline__ double weight(double Cw) const { return wp * Cw; }
    __device__ __forceinline__ double value(double f, double C) const
    {
#pragma clang fp contract(off)
        return f * wp * C;
    }
};
#endif

// 2^-(ws + 32): the FP32 map's scale back to x (unused in FP64)
__device__ __forceinline__ float map_scale(const DevConst* c) { return ldexpf(c->dscale32, -32); }

// LDS: table [d][N] (128-byte aligned), histogram [d][N][rep] (HIST only),
// then the block reduction's wave partials.
template <bool HIST>
__device__ __forceinline__ void sample(const SampleArgs& a, const double* __restrict__ params)
{
    extern __shared__ __align__(128) unsigned char smem[];
    const int N = a.N;
    const int dN = D * N;
    const size_t tab_bytes = (size_t(dN) * sizeof(tab_t) + 127) & ~size_t(127);
    const int rl2 = a.hrep_log2, rep = 1 << rl2;
    const int lrep = int(threadIdx.x) & (rep - 1);
    const size_t hist_bytes = HIST ? size_t(dN) * rep * sizeof(double) : 0;
    tab_t* tab = reinterpret_cast<tab_t*>(smem);
    double* hist = reinterpret_cast<double*>(smem + tab_bytes);
    double* red = reinterpret_cast<double*>(smem + tab_bytes + hist_bytes);

    const tab_t* gtab = static_cast<const tab_t*>(a.tab);
    for (int k = threadIdx.x; k < dN; k += blockDim.x) tab[k] = gtab[k];
    if constexpr (HIST)
        for (int k = threadIdx.x; k < dN * rep; k += blockDim.x) hist[k] = 0.0;
    __syncthreads();

    const BinConsts bc = bin_consts(N, a.cst);
    const double C = a.cst->C;  // N^d (FP32: times 2^(-ws d))
    const float ds = map_scale(a.cst);
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    double g1 = 0.0, g2 = 0.0;
    int ng = 0;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t k = uint64_t(threadIdx.x) * gridDim.x + blockIdx.x; k < a.n; k += stride) {
        Event ev;
        ev.run(tab, bc, a.e0 + k, a.t, a.ctr3, a.key0, a.key1, N, ds);
        const vegas_real f = vegas_integrand(ev.x, D, params);
        double v, v2;
        {
#pragma clang fp contract(off)
            v = ev.value(f, C);
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
        if constexpr (HIST) {
#pragma unroll
            for (int i = 0; i < D; ++i) lds_atomic_add(&(hist + (i * N << rl2))[(ev.b[i] << rl2) | lrep], v2);
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
    if constexpr (HIST) {
        double* slot = a.hslots + size_t((blockIdx.x >> 3) % kHistSlots) * dN;
        for (int k = threadIdx.x; k < dN; k += blockDim.x) {
            const int base = k << rl2;
            double h = 0.0;
            for (int r = 0; r < rep; ++r) h += hist[base + r];
            atomicAdd(&slot[k], h);
        }
    }
}

}  // namespace user
}  // namespace vegas

extern "C" __global__ __launch_bounds__(VEGAS_THREADS) void vegas_user_sample(vegas::SampleArgs a,
                                                                              const double* __restrict__ params)
{
    vegas::user::sample<true>(a, params);
}

extern "C" __global__ __launch_bounds__(VEGAS_THREADS) void vegas_user_sample_nohist(vegas::SampleArgs a,
                                                                                     const double* __restrict__ params)
{
    vegas::user::sample<false>(a, params);
}

// Per-event records b[d], delta[d], x[d], w, f (w = N^d prod W_b), widened
// to FP64, one event per thread; LDS holds the table.
extern "C" __global__ __launch_bounds__(256) void vegas_user_dump(vegas::DumpArgs a, const double* __restrict__ params)
{
    using namespace vegas;
    constexpr int D = user::D;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    using tab_t = user::tab_t;
    tab_t* tab = reinterpret_cast<tab_t*>(smem);
    const tab_t* gtab = static_cast<const tab_t*>(a.tab);
    for (int k = threadIdx.x; k < D * N; k += blockDim.x) tab[k] = gtab[k];
    __syncthreads();
    const BinConsts bc = user::bin_consts(N, a.cst);
    const double Cw = a.cst->Cw;
    const float ds = user::map_scale(a.cst);
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < a.n; k += stride) {
        user::Event ev;
        ev.run(tab, bc, a.e0 + k, a.t, a.ctr3, a.key0, a.key1, N, ds);
        double* row = a.out + k * size_t(3 * D + 2);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            row[i] = double(ev.b[i]);
            row[D + i] = ev.delta(i, bc);
            row[2 * D + i] = double(ev.x[i]);
        }
        row[3 * D] = ev.weight(Cw);
        row[3 * D + 1] = double(vegas_integrand(ev.x, D, params));
    }
}
