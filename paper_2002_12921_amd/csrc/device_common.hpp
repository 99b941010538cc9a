// Device building blocks of the Vegas event kernels: Philox4x32-10, exact
// binning, the piecewise-linear map, the integrands and block reductions.
#pragma once

#include "vegas_internal.hpp"

namespace vegas {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, sec. 3.2): ten rounds of
// two 32x32->64 multiplies whose halves are XOR-mixed with the other words
// and the key; the key advances by the Weyl constants between rounds.  The
// key and counter words 2..3 are uniform across a wave, so the key schedule
// stays in scalar registers.  Each 64-bit product is one v_mad_u64_u32 and
// each three-way XOR one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c).
struct U4 {
    uint32_t w[4];
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = uint64_t(c0) * 0xD2511F53u;
        const uint64_t p1 = uint64_t(c2) * 0xCD9E8D57u;
        const uint32_t n0 = xor3(uint32_t(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3(uint32_t(p0 >> 32), c3, k1);
        c1 = uint32_t(p1);
        c3 = uint32_t(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    U4 o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

// ---------------------------------------------------------------------------
// Precision policies.
struct P64 {
    using real = double;
    using tab_t = double2;
    static constexpr bool is64 = true;
};
struct P32 {
    using real = float;
    using tab_t = float2;
    static constexpr bool is64 = false;
};

__device__ __forceinline__ double exp_unit(double z) { return exp(z); }  // e^z
__device__ __forceinline__ float exp2_unit(float z) { return __builtin_amdgcn_exp2f(z); }

// The word k stands for y = (k + 1/2)/2^32.  yN = k N/2^32 + N/2^33 is exact
// in FP64 (at most 41 significant bits for N < 256), so the bin b = floor(yN)
// and delta = yN - b are exact: every precision bins every event alike.
__device__ __forceinline__ void bin_exact(uint32_t k, double nscale, double nhalf, int& b,
                                          double& delta)
{
    const double yn = fma(double(k), nscale, nhalf);
    b = int(yn);                            // truncation == floor for yn >= 0
    delta = __builtin_amdgcn_fract(yn);     // yn - floor(yn), exact
}

// Integrand constants of one problem, read once per thread into registers
// (they are uniform, so they normally live in scalar registers).
template <class P, int KIND, int DMAX>
struct EvalConsts {
    using real = typename P::real;
    real p1[DMAX], p2[DMAX];
    real kexp, wgroup, wlast;
    double nscale, nhalf, C, Cf, Cw;

    __device__ __forceinline__ void load(const DevConst* __restrict__ c)
    {
#pragma unroll
        for (int i = 0; i < DMAX; ++i) {
            p1[i] = P::is64 ? real(c->p1_64[i]) : real(c->p1_32[i]);
            p2[i] = P::is64 ? real(c->p2_64[i]) : real(c->p2_32[i]);
        }
        kexp = P::is64 ? real(c->kexp64) : real(c->kexp32);
        wgroup = real(c->wgroup32);
        wlast = real(c->wlast32);
        nscale = c->nscale;
        nhalf = c->nhalf;
        C = c->C;
        Cf = c->Cf;
        Cw = c->Cw;
    }
};

// Per-event evaluation shared by the sampling, dump and adjoint kernels.
// Computes, for the event's d uniforms, the bins, map, width product and the
// unnormalised integrand F; the event value is v = (double)(F*wp) * C.
// EXACT: d == DMAX, so no per-dimension guards are needed.
template <class P, int KIND, int DMAX, bool EXACT = false>
struct EventEval {
    using real = typename P::real;
    using tab_t = typename P::tab_t;

    int b[DMAX];      // bin of each dimension
    real x[DMAX];     // mapped point
    real del[DMAX];   // position inside the bin
    real wp;          // width product (scaled)
    real F;           // unnormalised integrand
    real s;           // Gaussian: sum (x_i - mu_i)^2

    __device__ __forceinline__ void run(const EvalConsts<P, KIND, DMAX>& c, const tab_t* __restrict__ tab,
                                        uint64_t e, uint32_t t, uint32_t ctr3, uint32_t key0,
                                        uint32_t key1, int d_rt, int N)
    {
        const int d = EXACT ? DMAX : d_rt;
        real w = real(1);
        real sa = real(0), sb = real(0);  // Gaussian / bimodal exponents; DISC: sum c (x-1)
        real den = real(1);               // PEAK: product of denominators
        bool inside = true;               // DISC: all x_i > a_i
        const uint32_t elo = uint32_t(e), ehi = uint32_t(e >> 32);
#pragma unroll
        for (int g = 0; g < DMAX / 4; ++g) {
            if (4 * g < d) {
                const U4 k = philox4x32_10(elo, ehi, t, ctr3 + uint32_t(g), key0, key1);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * g + q;
                    if (i < d) {
                        int bi;
                        double d64;
                        bin_exact(k.w[q], c.nscale, c.nhalf, bi, d64);
                        b[i] = bi;
                        const tab_t tb = (tab + i * N)[bi];
                        const real dl = real(d64);
                        const real xi = fma(dl, tb.y, tb.x);
                        del[i] = dl;
                        x[i] = xi;
                        w *= tb.y;
                        if constexpr (KIND == GAUSS) {
                            const real u = xi - c.p1[i];
                            sa = fma(u, u, sa);
                        } else if constexpr (KIND == BIMODAL) {
                            const real u = xi - c.p1[i];
                            const real v = xi - c.p2[i];
                            sa = fma(u, u, sa);
                            sb = fma(v, v, sb);
                        } else if constexpr (KIND == GENZ_DISC) {
                            inside = inside && (xi > c.p2[i]);
                            sa = fma(c.p1[i], xi - real(1), sa);
                        } else {  // GENZ_PEAK
                            const real u = xi - c.p2[i];
                            den *= fma(c.p1[i] * u, u, real(1));
                        }
                    }
                }
                if constexpr (!P::is64) {
                    // keep the FP32 width product near one: exact power-of-two rescale
                    w *= (4 * g + 4 <= d) ? c.wgroup : c.wlast;
                }
            }
        }
        wp = w;
        s = sa;
        if constexpr (KIND == GAUSS) {
            if constexpr (P::is64)
                F = exp_unit(-sa * c.kexp);
            else
                F = exp2_unit(-sa * c.kexp);
        } else if constexpr (KIND == BIMODAL) {
            if constexpr (P::is64)
                F = exp_unit(-sa * c.kexp) + exp_unit(-sb * c.kexp);
            else
                F = exp2_unit(-sa * c.kexp) + exp2_unit(-sb * c.kexp);
        } else if constexpr (KIND == GENZ_DISC) {
            // sa = sum c_i (x_i - 1) <= 0 (FP32: already times log2 e)
            if constexpr (P::is64)
                F = inside ? exp_unit(sa) : 0.0;
            else
                F = inside ? exp2_unit(sa) : 0.0f;
        } else {
            F = real(1) / den;
        }
    }

    __device__ __forceinline__ double value(const EvalConsts<P, KIND, DMAX>& c) const
    {
        return double(F * wp) * c.C;
    }
};

// ---------------------------------------------------------------------------
// Reductions.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Kahan step: s + (-c) tracks the running sum.
__device__ __forceinline__ void kahan_add(double& s, double& c, double v)
{
    const double y = v - c;
    const double t = s + y;
    c = (t - s) - y;
    s = t;
}

// Neumaier step: the sum is s + c.
__device__ __forceinline__ void neumaier_add(double& s, double& c, double v)
{
    const double t = s + v;
    if (fabs(s) >= fabs(v))
        c += (s - t) + v;
    else
        c += (v - t) + s;
    s = t;
}

// Block (kBlock threads) sum of one double; result valid in thread 0.
// red must hold kBlock/64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kBlock / 64; ++k) t += red[k];
    }
    __syncthreads();
    return t;
}

__device__ __forceinline__ void lds_atomic_add(double* p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

}  // namespace vegas
