// Device building blocks of the Vegas event kernels: Philox4x32-10, exact
// binning, the piecewise-linear map, the integrands and block reductions.
#pragma once

#include "vegas_internal.hpp"

namespace vegas {

// Type selection (std::conditional, which the runtime compiler lacks).
template <bool B, class T, class F>
struct pick_type {
    using type = T;
};
template <class T, class F>
struct pick_type<false, T, F> {
    using type = F;
};

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
// Precision policies and grid-table entry types.
//
// FP64: table entry (E_b - c, E_{b+1} - E_b) for the integrand's centre c, so
//   u = x - c = fma(delta, width, E_b - c) is one fma (x itself is not formed;
//   the centre is 0 for user integrands, whose table holds E_b).
// FP32: the map works on u' = (x - c) S with S = 2^(ws + 32).  With
//   delta = (lo + h)/2^32 (see bin_words) and W = RN32(width), the table entry is
//     (RN32((E_b - c + h W / 2^32) S), W 2^ws),
//   so u' = RN32(lo) (W 2^ws) + first entry is one int-to-float convert and one
//   FP32 fma: the convert rounds lo exactly as RN32(delta) would (delta itself
//   is never formed), the offset from the integrand's centre c makes u carry
//   rounding relative to u rather than to x, the factor 2^ws keeps the width
//   product near one, and the integrand's constants absorb S^-1, S^-2 exactly.
//   The bimodal integrand has two centres: (cA entry, cB entry, W 2^ws, 0).
struct P64 {
    using real = double;
    static constexpr bool is64 = true;
};
struct P32 {
    using real = float;
    static constexpr bool is64 = false;
};

template <class P, int KIND>
struct TabEntry {
    using type = float2;
};
template <int KIND>
struct TabEntry<P64, KIND> {
    using type = double2;
};
template <>
struct TabEntry<P32, BIMODAL> {
    using type = float4;
};

__device__ __forceinline__ double exp_unit(double z) { return exp(z); }  // e^z
__device__ __forceinline__ float exp2_unit(float z) { return __builtin_amdgcn_exp2f(z); }

// The word k stands for y = (k + 1/2)/2^32, so yN = (kN + N/2) / 2^32.  With
// P = kN + floor(N/2), one 32x32+32 -> 64-bit multiply-add, yN = (P + h)/2^32
// where h = 1/2 for odd N and 0 for even N; since P + h never reaches the next
// multiple of 2^32, the bin b = floor(yN) is the high word of P and
// delta = yN - b = (lo + h) / 2^32, lo the low word.  The bin is exact in
// every precision and FP64 gets delta exactly; the FP32 map carries RN32(lo).
struct BinConsts {
    uint32_t mul, add;  // N, floor(N/2)
    double h64;         // h / 2^32
    double s32;         // 2^-32, read from memory: in a scalar register the FP64
                        // fma delta = lo 2^-32 + h64 needs no copy of its addend
};

__device__ __forceinline__ void bin_words(uint32_t k, const BinConsts& bc, int& b, uint32_t& lo)
{
    const uint64_t P = uint64_t(k) * bc.mul + bc.add;
    b = int(uint32_t(P >> 32));
    lo = uint32_t(P);
}

// Integrand constants of one problem, read once per thread into registers
// (they are uniform, so they normally live in scalar registers).
template <class P, int KIND, int DMAX>
struct EvalConsts {
    using real = typename P::real;
    real p1[DMAX], p2[DMAX];
    double c64[DMAX];   // FP32 path, DISC: c_i / S (exponent summed in FP64, d > 8)
    float c32[DMAX];    // FP32 path, DISC: RN32(c_i / S) (exponent summed in FP32, d <= 8)
    real kexp, dscale;  // dscale: FP32 path, 1/S = 2^-(ws + 32)
    double k2;          // FP32 path: log2(e)/(a S)^2 (GAUSS, BIMODAL), log2(e) (DISC)
    BinConsts bc;
    double C, Cf, Cw;
    // DISC: x_i > a_i exactly when the event's binning word k_i >= K_i; lane
    // l holds K_l (l < d), read with v_readlane (which ignores EXEC, so it is
    // safe in the partial last pass); never: some K_i = 2^32, no event is
    // inside
    uint32_t kv;
    bool never;

    // thr_g: the d thresholds T_i of the discontinuous integrand in
    // P = b 2^32 + lo (disc_threshold; other kinds: unused, may be null).
    // Called by every thread of the wave (it takes a ballot).
    __device__ __forceinline__ void load(const DevConst* __restrict__ c, const uint64_t* __restrict__ thr_g, int d)
    {
        // only what the kernel's precision and integrand read (scalar registers
        // are scarce); the FP32 path works on u S, S = 2^(ws + 32), so its
        // constants take the matching powers of 1/S (exact)
        const double ds = double(c->dscale32) * 0x1p-32, ds2 = ds * ds;
#pragma unroll
        for (int i = 0; i < DMAX; ++i) {
            p1[i] = real(0);
            p2[i] = real(0);
            c64[i] = 0.0;
            c32[i] = 0.0f;
            if constexpr (P::is64) {
                // the centres are in the table: GENZ c (DISC) or c^2 (PEAK),
                // BIMODAL muB - muA
                if constexpr (KIND == GENZ_DISC || KIND == GENZ_PEAK) p1[i] = c->p1_64[i];
                if constexpr (KIND == BIMODAL) p2[i] = c->p2_64[i];
            } else {
                if constexpr (KIND == GENZ_PEAK) p1[i] = real(sqrt(c->p1_64[i]) * ds);  // c_i / S
                if constexpr (KIND == GENZ_DISC) {
                    c64[i] = c->p1_64[i] * ds;
                    c32[i] = float(c64[i]);
                }
            }
        }
        kexp = P::is64 ? real(c->kexp64) : real(0);
        k2 = (P::is64 || KIND == GENZ_DISC) ? c->kexp2_64 : c->kexp2_64 * ds2;
        dscale = real(ds);
        const uint32_t N = uint32_t(c->n_bins);
        bc.mul = N;
        bc.add = N >> 1;
        bc.h64 = (N & 1u) ? 0x1p-33 : 0.0;
        bc.s32 = c->two_m32;
        C = c->C;
        Cf = c->Cf;
        Cw = c->Cw;
        kv = 0;
        never = false;
        if constexpr (KIND == GENZ_DISC) {
            // P = k N + floor(N/2) grows with k, so P >= T exactly when
            // k >= K = ceil((T - floor(N/2)) / N) (0 when T <= floor(N/2))
            const int lane = int(threadIdx.x & 63u);
            uint64_t K = 0;
            if (lane < d) {
                const uint64_t T = thr_g[lane], off = N >> 1;
                K = T <= off ? 0 : (T - off + N - 1) / N;
            }
            never = __ballot(K > 0xffffffffull) != 0;
            kv = uint32_t(K);
        }
    }
};

// Per-event evaluation shared by the sampling, dump and adjoint kernels.
// Computes, for the event's d uniforms, the bins, the offsets u_i = x_i - c_i
// from the integrand's centres, the width product wp and the integrand's
// significand F; the event value is v = ldexp(F * wp, ew + fe) * C
// (FP64: ew = fe = 0).  EXACT: d == DMAX, so no per-dimension guards are needed.
template <class P, int KIND, int DMAX, bool EXACT = false>
struct EventEval {
    using real = typename P::real;
    using tab_t = typename TabEntry<P, KIND>::type;

    int b[DMAX];      // bin of each dimension
    real u[DMAX];     // x_i - centre_i (GAUSS, BIMODAL: mu / muA; DISC, PEAK: a_i); FP32: times S
    real del[DMAX];   // FP64: position inside the bin; FP32: RN32(lo)
    real wp;          // width product (FP32: scaled, see ew)
    real F;           // integrand significand
    real s;           // GAUSS: sum u_i^2
    double s64;       // GAUSS: sum u_i^2 as accumulated (FP64 in both paths; FP32: of u S)
    int ew;           // FP32: binary exponent taken out of the width product
    int fe;           // FP32: binary exponent of the integrand (f ~ 2^fe F)

    __device__ __forceinline__ void run(const EvalConsts<P, KIND, DMAX>& c, const tab_t* __restrict__ tab,
                                        uint64_t e, uint32_t t,
                                        uint32_t ctr3, uint32_t key0, uint32_t key1, int d_rt, int N)
    {
        // every fused multiply-add here is an explicit fma(): nothing else is
        // contracted, so all kernel variants round the same way
#pragma clang fp contract(off)
        const int d = EXACT ? DMAX : d_rt;
        // the FP32 path sums the exponent in FP32 up to d = 8 (error <= d 2^-24
        // of the exponent) and in FP64 beyond, where that grows past the
        // method's tolerance
        constexpr bool kQ32 = !P::is64 && DMAX <= 8;
        using q_t = typename pick_type<kQ32, float, double>::type;
        real w = real(1);
        real sa = real(0), sb = real(0);  // FP64 path: GAUSS/BIMODAL sums of squares; DISC: sum c u
        q_t qa = q_t(0), qb = q_t(0);     // FP32 path: the same sums
        real den = real(1);               // PEAK: product of denominators
        bool inside = true;               // DISC: all x_i > a_i
        int ewl = 0;                      // FP32: exponent taken out of w
        const uint32_t elo = uint32_t(e), ehi = uint32_t(e >> 32);
        // one Philox call per group of four dimensions (the last group may be
        // partial: DMAX need not be a multiple of 4)
#pragma unroll
        for (int g = 0; g < (DMAX + 3) / 4; ++g) {
            if (4 * g < d) {
                const U4 k = philox4x32_10(elo, ehi, t, ctr3 + uint32_t(g), key0, key1);
                // the group's four bins and table entries first, so that its
                // LDS reads are in flight together before any is used
                int bq[4];
                uint32_t loq[4];
                tab_t tq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * g + q;
                    if (i < d) {
                        bin_words(k.w[q], c.bc, bq[q], loq[q]);
                        tq[q] = (tab + i * N)[bq[q]];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * g + q;
                    if (i < d) {
                        const int bi = bq[q];
                        const uint32_t lo = loq[q];
                        b[i] = bi;
                        const tab_t tb = tq[q];
                        real ui, ubi = real(0), width;
                        real dl;
                        if constexpr (P::is64) {
                            dl = fma(double(lo), c.bc.s32, c.bc.h64);
                            width = tb.y;
                            ui = fma(dl, tb.y, tb.x);
                            if constexpr (KIND == BIMODAL) ubi = ui - c.p2[i];  // p2 = muB - muA
                        } else if constexpr (KIND == BIMODAL) {
                            dl = float(lo);
                            width = tb.z;
                            ui = fma(dl, tb.z, tb.x);
                            ubi = fma(dl, tb.z, tb.y);
                        } else {
                            dl = float(lo);
                            width = tb.y;
                            ui = fma(dl, tb.y, tb.x);
                        }
                        del[i] = dl;
                        u[i] = ui;
                        w *= width;
                        if constexpr (KIND == GAUSS) {
                            if constexpr (P::is64)
                                sa = fma(ui, ui, sa);
                            else  // (u^2 of an FP32 u is exact in FP64)
                                qa = fma(q_t(ui), q_t(ui), qa);
                        } else if constexpr (KIND == BIMODAL) {
                            if constexpr (P::is64) {
                                sa = fma(ui, ui, sa);
                                sb = fma(ubi, ubi, sb);
                            } else {
                                qa = fma(q_t(ui), q_t(ui), qa);
                                qb = fma(q_t(ubi), q_t(ubi), qb);
                            }
                        } else if constexpr (KIND == GENZ_DISC) {
                            // x_i > a_i as the FP64 x decides it: one integer
                            // comparison of the binning word with K_i, in both
                            // precisions
                            inside = inside & (k.w[q] >= uint32_t(__builtin_amdgcn_readlane(int(c.kv), i)));
                            if constexpr (P::is64)
                                sa = fma(c.p1[i], ui, sa);
                            else if constexpr (kQ32)
                                qa = fma(c.c32[i], ui, qa);
                            else
                                qa = fma(c.c64[i], double(ui), qa);
                        } else {  // GENZ_PEAK: (c u)^2 + 1
                            if constexpr (P::is64) {
                                den *= fma(c.p1[i] * ui, ui, real(1));  // p1 = c^2
                            } else {
                                const real cu = c.p1[i] * ui;  // p1 = c / S, ui = u S
                                den *= fma(cu, cu, real(1));
                            }
                        }
                    }
                }
                if constexpr (!P::is64) {
                    // every 8 dimensions move w's exponent into ew (no FP32 under/overflow)
                    if ((g & 1) == 1 && 4 * g + 4 < d) {
                        int e2;
                        w = frexpf(w, &e2);
                        ewl += e2;
                    }
                }
            }
        }
        if constexpr (KIND == GENZ_DISC) inside = inside && !c.never;
        wp = w;
        s = sa;
        s64 = P::is64 ? double(sa) : double(qa);
        ew = ewl;
        if constexpr (P::is64) {
            fe = 0;
            if constexpr (KIND == GAUSS)
                F = exp_unit(-sa * c.kexp);
            else if constexpr (KIND == BIMODAL)
                F = exp_unit(-sa * c.kexp) + exp_unit(-sb * c.kexp);
            else if constexpr (KIND == GENZ_DISC)
                F = inside ? exp_unit(sa) : 0.0;  // sa = sum c (x - a)
            else
                F = real(1) / den;
        } else {
            // FP32 significand, FP64 exponent: with the exponent A (base 2)
            // formed in FP64, m = floor(A) and F = 2^(m - A) in (1/2, 1] in
            // FP32, so f = 2^-m F Cf keeps FP64 range
            s = float(qa);
            if constexpr (KIND == GAUSS) {
                const double arg = double(qa) * c.k2;
                const double m = floor(arg);
                F = exp2_unit(float(m - arg));
                fe = -int(m);
            } else if constexpr (KIND == BIMODAL) {
                const double aa = double(qa) * c.k2, ab = double(qb) * c.k2;
                const double m = floor(fmin(aa, ab));
                F = exp2_unit(float(fmax(m - aa, -200.0))) + exp2_unit(float(fmax(m - ab, -200.0)));
                fe = -int(m);
            } else if constexpr (KIND == GENZ_DISC) {
                const double arg = -double(qa) * c.k2;  // qa = sum c (x - a) >= 0 inside
                const double m = floor(arg);
                F = inside ? exp2_unit(float(m - arg)) : 0.0f;
                fe = -int(m);
            } else {
                F = 1.0f / den;
                fe = 0;
            }
        }
    }

    // The product is rounded as written (no fusion into a following add), so
    // every kernel variant accumulates the same rounded v.
    __device__ __forceinline__ double value(const EvalConsts<P, KIND, DMAX>& c) const
    {
#pragma clang fp contract(off)
        if constexpr (P::is64)
            return F * wp * c.C;
        else
            return ldexp(double(F * wp), ew + fe) * c.C;
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

// Event kernels add kGroup events per thread in plain FP64, then fold the
// group's sums into Kahan-compensated S1, S2.
constexpr int kGroup = 8;

// Kahan step: s + (-c) tracks the running sum.
__device__ __forceinline__ void kahan_add(double& s, double& c, double v)
{
    const double y = v - c;
    const double t = s + y;
    c = (t - s) - y;
    s = t;
}

// Branch-free compensated step (Knuth's TwoSum): the sum is s + c.
__device__ __forceinline__ void twosum_add(double& s, double& c, double v)
{
    const double t = s + v;
    const double bp = t - s;
    c += (s - (t - bp)) + (v - bp);
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

// Block sum of one double (blockDim.x a multiple of 64); result valid in
// thread 0.  red must hold blockDim.x/64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = int(blockDim.x) >> 6;
        for (int k = 0; k < nw; ++k) t += red[k];
    }
    __syncthreads();
    return t;
}

// Fixed-order sum of the (d + 1)-column rows part[rows][d + 1] of an
// adjoint: one wave per column j (and j + 16, ...), lane l adding rows l,
// l + 64, ... in order with two-sums, then an exact two-sum butterfly across
// the wave (the same pair on every lane); column j times `scale` goes to
// out[j], in FP64 or rounded once to FP32 (out_fp32).  Called by a whole
// block of kMergeThreads threads.
__device__ __forceinline__ void adjoint_merge_block(const double* part, int rows, int d, double scale, void* out,
                                                    int out_fp32)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j <= d; j += kMergeThreads / 64) {
        double s = 0.0, c = 0.0;
        for (int r = lane; r < rows; r += 64) twosum_add(s, c, part[size_t(r) * (d + 1) + j]);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double s2 = __shfl_xor(s, o, 64), c2 = __shfl_xor(c, o, 64);
            twosum_add(s, c, s2);
            c += c2;
        }
        if (lane == 0) {
            const double g = (s + c) * scale;
            if (out_fp32)
                static_cast<float*>(out)[j] = float(g);
            else
                static_cast<double*>(out)[j] = g;
        }
    }
}

// Inclusive prefix sum over the 64 lanes of a wave (lane order).
__device__ __forceinline__ double wave_inclusive_scan(double v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// Running maximum over the 64 lanes of a wave (lane order).
__device__ __forceinline__ double wave_inclusive_max(double v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(v, off, 64);
        if (lane >= off) v = fmax(v, o);
    }
    return v;
}

__device__ __forceinline__ void lds_atomic_add(double* p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

}  // namespace vegas
