// Device routines shared by the single-problem and batched reduction kernels:
// the statistics of one iteration, the grid tables and the refinement.
#pragma once

#include "device_common.hpp"

namespace vegas {

// Statistics of one iteration (Lepage 1978 sec. 3): I_t = S1/M and the
// variance of that mean, var_t = (S2/M - I_t^2)/(M - 1).  The iteration is
// recorded (unless NO_RECORD: then it only becomes the last iteration's
// estimate); the combination over recorded iterations runs in k_combine.
__device__ static void finish_iteration(const MergeArgs& a, double S1, double S2)
{
    const double M = a.M;
    const double I = S1 / M;
    const double var = (S2 / M - I * I) / (M - 1.0);
    const bool ok = isfinite(I) && isfinite(var);
    if (a.last_out) {
        a.last_out[0] = I;
        a.last_out[1] = sqrt(var);
    }
    DevResult* R = a.result;
    if (a.flags & MERGE_NO_RECORD) {
        R->last_integral = I;
        R->last_var = var;
        return;
    }
    const int rec = a.rec_idx;
    a.records[2 * rec] = I;
    a.records[2 * rec + 1] = var;
    a.rec_flag[rec] = (ok && !(a.flags & MERGE_NO_COMBINE)) ? 1 : 0;
    R->last_integral = I;
    R->last_var = var;
    R->n_iter = rec + 1;
    R->n_events += int64_t(M);
    if (!ok) R->n_nonfinite += 1;
}

// Grid tables of dimension i from its edges E[0..N] (any address space).
//   FP64: (E_b - cA, E_{b+1} - E_b), cA the integrand's centre (0 for user
//         integrands); the event kernel forms x - cA with one fma
//   FP32: with W = RN32(E_{b+1} - E_b), S = 2^(ws + 32) and g = E_b + h W / 2^32
//         (h = 1/2 for odd N, else 0),
//         (RN32((g - cA) S), [RN32((g - cB) S),] W 2^ws)
//   The event kernel forms (x - c) S = RN32(lo) W 2^ws + first entry.
__device__ __forceinline__ void write_table_entry(int i, int b, double lo, double hi, double cA, double cB,
                                                  float dscale32, int kind, int N, double2* tab64, float* tab32)
{
    const double sw = 1.0 / double(dscale32);  // 2^ws
    const double S = sw * 0x1p32;
    const double h = (N & 1) ? 0x1p-33 : 0.0;     // h / 2^32
    const double w = hi - lo;
    tab64[size_t(i) * N + b] = make_double2(lo - cA, w);
    const double W = double(float(w));
    const double g = lo + h * W;
    const float Ws = float(W * sw);
    if (kind == BIMODAL) {
        reinterpret_cast<float4*>(tab32)[size_t(i) * N + b] =
            make_float4(float((g - cA) * S), float((g - cB) * S), Ws, 0.0f);
    } else {
        reinterpret_cast<float2*>(tab32)[size_t(i) * N + b] = make_float2(float((g - cA) * S), Ws);
    }
}

__device__ __forceinline__ void write_table_entry(int i, int b, double lo, double hi, const DevConst* __restrict__ c,
                                                  int kind, int N, double2* tab64, float* tab32)
{
    write_table_entry(i, b, lo, hi, c->cA64[i], c->cB64[i], c->dscale32, kind, N, tab64, tab32);
}

// The discontinuous integrand (Eq. genzdisc) is zero unless x_i > a_i in
// every dimension, a decision the method takes on x = E_b + delta (E_{b+1} -
// E_b) in FP64.  The event's bin and position come from the 64-bit integer
// P = b 2^32 + lo (delta = (lo + h)/2^32, see bin_words), and x, evaluated
// in that order in FP64, never decreases as P grows: within a bin every
// operation is monotone, and the largest delta, 1 - 2^-33, keeps the exact
// value below E_{b+1} by more than the two roundings can add, so no x of a
// bin exceeds the next bin's lower edge.  Hence x > a holds exactly when
// P >= T for the smallest such P, which is found here once per grid (a
// bisection over lo in the bin that holds a), and the event kernels, FP64
// and FP32 alike, decide with one integer comparison what the FP64 x would.
// The threshold within bin b (edges Eb <= a < Eb1) of a grid of N bins.
__device__ static uint64_t disc_bin_threshold(double Eb, double Eb1, int b, int N, double a)
{
#pragma clang fp contract(off)
    const double w = Eb1 - Eb;
    const double h = (N & 1) ? 0.5 : 0.0;
    uint64_t lo = 0, hi = uint64_t(1) << 32;  // hi: no event of bin b lies above a
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const double x = Eb + ((double(mid) + h) * 0x1p-32) * w;
        if (x > a)
            hi = mid;
        else
            lo = mid + 1;
    }
    return (uint64_t(b) << 32) + lo;
}

__device__ static uint64_t disc_threshold(const double* E, int N, double a)
{
    int b = 0;  // the bin holding a: the last b with E_b <= a (E_0 = 0 <= a < 1 = E_N)
    for (int k = 1; k < N; ++k)
        if (E[k] <= a) b = k;
    return disc_bin_threshold(E[b], E[b + 1], b, N, a);
}

__device__ static void write_tables(int i, const double* E, const DevConst* __restrict__ c, int kind,
                                    int N, double2* tab64, float* tab32, uint64_t* thr)
{
    for (int b = threadIdx.x; b < N; b += blockDim.x) write_table_entry(i, b, E[b], E[b + 1], c, kind, N, tab64, tab32);
    if (kind == GENZ_DISC && threadIdx.x == 0) thr[i] = disc_threshold(E, N, c->cA64[i]);
}

// Scale of the FP32 table's widths: 2^-ws with ws = round(log2 N), so the
// product of d scaled widths stays near one.
__device__ __forceinline__ float width_scale32(int N) { return ldexpf(1.0f, -int(rint(log2(double(N))))); }

// The table centres of dimension i from the raw parameters q (layouts of
// vegas_desc.params): GAUSS mu_i; BIMODAL muA_i and muB_i; Genz a_i; USER 0.
__device__ __forceinline__ void table_centres(int kind, int d, int i, const double* q, double& cA, double& cB)
{
    cA = 0.0;
    cB = 0.0;
    if (kind == GAUSS || kind == BIMODAL) cA = q[1 + i];
    if (kind == BIMODAL) cB = q[1 + d + i];
    if (kind == GENZ_DISC || kind == GENZ_PEAK) cA = q[d + i];
}

// Damping of the refinement: r(s) = ((s - 1)/ln s)^alpha, r(0) = 0, r(1) = 1.
// The usual exponents take a square root and a product instead of pow
// (within two roundings of it).
__device__ static double damp(double s, double alpha)
{
    if (s == 0.0) return 0.0;
    if (s == 1.0) return 1.0;
    const double x = (s - 1.0) / log(s);
    if (alpha == 1.5) return x * sqrt(x);
    if (alpha == 1.0) return x;
    if (alpha == 0.5) return sqrt(x);
    if (alpha == 2.0) return x * x;
    return pow(x, alpha);
}

// Refinement of dimension i from its histogram h[0..N-1] (LDS), by the whole
// block (Lepage 1978 sec. 3, continuous rebinning): smooth with a 3-point
// mean, normalise, damp, then put new edge k where the cumulative damped
// weight, spread uniformly over each old bin, first reaches k/N of its total.
// The smoothing and the damping (a log and a power in FP64) take one bin per
// thread; wave 0 forms the two totals and the cumulative weights
// C_b = r_0 + ... + r_b (four bins per lane, then a scan across lanes; a
// running maximum keeps C non-decreasing under rounding); every thread then
// places its new edges by bisection on C.  Bins with r = 0 are never chosen:
// the first b with C_b >= level has C_{b-1} < level <= C_b.
// Needs blockDim.x > N; Eo holds the current edges (LDS, filled by the
// caller before a barrier).
__device__ static void refine_dim(const MergeArgs& a, int i, const double* h, const double* Eo)
{
    const int N = a.N;
    __shared__ double En[kMaxBins + 1], Cs[kMaxBins + 1];
    __shared__ double tot[2];
    double* E = a.edges + size_t(i) * (N + 1);
    const int t = threadIdx.x;
    if (t < N) {
        const double l = t > 0 ? h[t - 1] : 0.0;
        const double r = t < N - 1 ? h[t + 1] : 0.0;
        double sm;
        if (t == 0)
            sm = (h[t] + r) / 2.0;
        else if (t == N - 1)
            sm = (l + h[t]) / 2.0;
        else
            sm = (l + h[t] + r) / 3.0;
        Cs[t] = sm;
    }
    __syncthreads();
    if (t < 64) {
        double th = 0.0, ts = 0.0;
        for (int b = t; b < N; b += 64) {
            th += h[b];
            ts += Cs[b];
        }
        th = wave_sum(th);
        ts = wave_sum(ts);
        if (t == 0) {
            tot[0] = th;
            tot[1] = ts;
        }
    }
    __syncthreads();
    // an empty histogram, or one whose totals are not finite (an overflowing
    // or NaN integrand): the grid and its tables stay
    if (!(tot[0] > 0.0 && tot[0] <= __DBL_MAX__ && tot[1] > 0.0 && tot[1] <= __DBL_MAX__)) return;
    if (t < N) Cs[t] = damp(Cs[t] / tot[1], a.alpha);
    __syncthreads();
    if (t < 64) {
        const int lane = t;
        double c[4];
        double run = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = 4 * lane + q;
            run += b < N ? Cs[b] : 0.0;
            c[q] = run;
        }
        const double excl = wave_inclusive_scan(run) - run;
        double mx = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = fmax(excl + c[q], mx);
            mx = c[q];
        }
        const double lane_max = wave_inclusive_max(mx);
        const double prev = __shfl_up(lane_max, 1, 64);
        const double floor_ = lane > 0 ? prev : 0.0;
        // each lane reads and writes only its own four bins
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = 4 * lane + q;
            if (b < N) Cs[b] = fmax(c[q], floor_);
        }
    }
    __syncthreads();
    const double R = Cs[N - 1];
    for (int k = t; k <= N; k += blockDim.x) {
        double e;
        if (k == 0 || k == N) {
            e = Eo[k];
        } else {
            const double level = double(k) * R / double(N);
            int lo = 0, hi = N - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (Cs[mid] >= level)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            const int b = lo;
            const double A = b > 0 ? Cs[b - 1] : 0.0;
            e = Eo[b] + (level - A) / (Cs[b] - A) * (Eo[b + 1] - Eo[b]);
        }
        En[k] = e;
        E[k] = e;
    }
    __syncthreads();
    write_tables(i, En, a.cst, a.kind, N, a.tab64, a.tab32, a.thr);
}

// The same refinement for N <= 64 by one wave (lane b holds bin b's value hb
// and the edges Eb = E_b, Eb1 = E_{b+1}), with no barrier: neighbours for the
// smoothing, the totals, the cumulative weights and the searches all go
// through cross-lane exchanges.  Each new interior edge k = lane is placed by
// a branch-free lower-bound search (six probes) for the first bin whose C
// reaches k R / N.  Called by a whole wave.
__device__ static void refine_dim_wave(const MergeArgs& a, int i, double hb, double Eb, double Eb1)
{
    const int N = a.N, b = threadIdx.x & 63;
    const bool in = b < N;
    if (!in) hb = 0.0;
    const double hl = __shfl_up(hb, 1, 64), hr = __shfl_down(hb, 1, 64);
    double sm = 0.0;
    if (in) {
        if (b == 0)
            sm = (hb + hr) / 2.0;
        else if (b == N - 1)
            sm = (hl + hb) / 2.0;
        else
            sm = (hl + hb + hr) / 3.0;
    }
    const double th = wave_sum(hb), ts = wave_sum(sm);
    // empty, or not finite (an overflowing or NaN integrand): the grid and its tables stay
    if (!(th > 0.0 && th <= __DBL_MAX__ && ts > 0.0 && ts <= __DBL_MAX__)) return;
    const double r = in ? damp(sm / ts, a.alpha) : 0.0;
    const double C = wave_inclusive_max(wave_inclusive_scan(r));  // non-decreasing under rounding
    const double R = __shfl(C, N - 1, 64);
    // new edge k = b (only 1 <= k <= N - 1 is used): lower bound of level in C
    const double level = double(b) * R / double(N);
    int pos = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int probe = pos + step - 1;
        const double cp = __shfl(C, probe < 63 ? probe : 63, 64);
        if (probe < N && cp < level) pos += step;
    }
    const double Am = __shfl(C, pos > 0 ? pos - 1 : 0, 64);
    const double A = pos > 0 ? Am : 0.0;
    const double Cp = __shfl(C, pos, 64);
    const double Ep = __shfl(Eb, pos, 64), Ep1 = __shfl(Eb1, pos, 64);
    const double e = Ep + (level - A) / (Cp - A) * (Ep1 - Ep);
    double* E = a.edges + size_t(i) * (N + 1);
    if (b >= 1 && b <= N - 1) E[b] = e;
    // tables of bin b: lower edge (new edge b, or the fixed E_0), upper edge
    // (new edge b + 1 from the next lane, or the fixed E_N)
    const double up = __shfl_down(e, 1, 64);
    const double lo = b == 0 ? Eb : e;
    const double hi = b == N - 1 ? Eb1 : up;
    if (in) write_table_entry(i, b, lo, hi, a.cst, a.kind, N, a.tab64, a.tab32);
    if (a.kind == GENZ_DISC) {
        // the bin holding a_i is the count of interior edges at or below it
        const double th = a.cst->cA64[i];
        const int bth = __popcll(__ballot(b >= 1 && b <= N - 1 && e <= th));
        const double El = __shfl(lo, bth, 64), Eu = __shfl(hi, bth, 64);
        if (b == 0) a.thr[i] = disc_bin_threshold(El, Eu, bth, N, th);
    }
}

// Stand-alone refinement of dimension i by the calling block from h (LDS):
// one wave for N <= 64, the whole block otherwise.
__device__ static inline void refine_any(const MergeArgs& a, int i, const double* h, const double* Eo)
{
    if (a.N <= 64) {
        if (threadIdx.x < 64) {
            const int b = threadIdx.x;
            refine_dim_wave(a, i, b < a.N ? h[b] : 0.0, b <= a.N ? Eo[b] : 0.0, b < a.N ? Eo[b + 1] : 0.0);
        }
        return;
    }
    refine_dim(a, i, h, Eo);
}

// One column group of the reduction (group 0: S1, S2; group 1+i: the
// histogram of dimension i): the partial rows are summed in a fixed order,
// folded into the chunk accumulator (when there is one), and at the end of
// the iteration the group records the statistics or refines its dimension.
// Histogram groups (when the rows carry H, as in batches): wave w adds rows
// w, w + 16, ... (lane = column, so each load instruction reads consecutive
// columns of one row), 32 loads in flight, with two-sums.  When the event
// kernel accumulated H in slots instead, the group adds the slots.  Group 0 spreads its rows over all lanes and folds
// each wave with a butterfly.  After one barrier wave 0 adds the 16 wave
// partials in order.  For N <= 64 wave 0 then refines with the column values
// still in its registers.
__device__ static void merge_group(const MergeArgs& a, const int g)
{
    const int ncol = g == 0 ? 2 : a.N;
    const int off = g == 0 ? 0 : 2 + (g - 1) * a.N;
    if (g > 0 && (a.flags & MERGE_NO_HIST)) {
        // an iteration without histograms: its histogram row reads zero
        if (a.flags & MERGE_END)
            for (int k = threadIdx.x; k < ncol; k += blockDim.x) a.last[off + k] = 0.0;
        return;
    }
    constexpr int kWaves = kMergeThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double ws_s[kWaves][kMaxBins + 1], ws_c[kWaves][kMaxBins + 1];
    __shared__ double fin[kMaxBins + 1], Eo[kMaxBins + 1];
    const bool end = a.flags & MERGE_END;
    const bool refine = end && (a.flags & MERGE_REFINE) && g > 0;
    const bool wave_refine = refine && a.N <= 64;
    // the edges the refinement needs, fetched while the rows are summed
    double Eb = 0.0, Eb1 = 0.0;
    if (wave_refine && wave == 0) {
        const double* E = a.edges + size_t(g - 1) * (a.N + 1);
        Eb = lane <= a.N ? E[lane] : 0.0;
        Eb1 = lane < a.N ? E[lane + 1] : 0.0;
    } else if (refine && !wave_refine && int(threadIdx.x) <= a.N) {
        Eo[threadIdx.x] = a.edges[size_t(g - 1) * (a.N + 1) + threadIdx.x];
    }
    if (g > 0 && a.hslots) {
        // histogram accumulated by the event kernel in kHistSlots slots (over
        // every chunk of the iteration): at its end, add the slots in order,
        // clear them for the next iteration, record, refine
        if (!end) return;
        const size_t dN = size_t(a.d) * a.N;
        double mine = 0.0;
        for (int col = threadIdx.x; col < ncol; col += blockDim.x) {
            double* h = a.hslots + size_t(g - 1) * a.N + col;
            double v[kHistSlots];
#pragma unroll
            for (int q = 0; q < kHistSlots; ++q) v[q] = h[q * dN];
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < kHistSlots; ++q) {
                sum += v[q];
                h[q * dN] = 0.0;
            }
            a.last[off + col] = sum;
            fin[col] = sum;
            if (col == int(threadIdx.x)) mine = sum;
        }
        if (!refine) return;
        if (wave_refine) {
            // columns 0..N-1 are lanes 0..N-1 of wave 0
            if (wave == 0) refine_dim_wave(a, g - 1, mine, Eb, Eb1);
            return;
        }
        __syncthreads();
        refine_dim(a, g - 1, fin, Eo);
        return;
    }
    if (g == 0) {
        // S1, S2: lane pairs take rows (thread t: row lane t / 2, column t % 2),
        // then an exact two-sum butterfly over the pairs of the wave
        const int col = lane & 1;
        double s = 0.0, c = 0.0;
        for (int r = int(threadIdx.x) >> 1; r < a.rows; r += kMergeThreads / 2)
            twosum_add(s, c, a.partials[size_t(r) * a.rstride + col]);
#pragma unroll
        for (int o = 2; o < 64; o <<= 1) {
            const double s2 = __shfl_xor(s, o, 64), c2 = __shfl_xor(c, o, 64);
            twosum_add(s, c, s2);
            c += c2;
        }
        if (lane < 2) {
            ws_s[wave][col] = s;
            ws_c[wave][col] = c;
        }
    }
    for (int col = lane; g > 0 && col < ncol; col += 64) {
        const double* base = a.partials + off + col;
        double s = 0.0, c = 0.0;
        int r = wave;
        for (; r + 31 * kWaves < a.rows; r += 32 * kWaves) {
            double v[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) v[u] = base[size_t(r + u * kWaves) * a.rstride];
#pragma unroll
            for (int u = 0; u < 32; ++u) twosum_add(s, c, v[u]);
        }
        for (; r + 7 * kWaves < a.rows; r += 8 * kWaves) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = base[size_t(r + u * kWaves) * a.rstride];
#pragma unroll
            for (int u = 0; u < 8; ++u) twosum_add(s, c, v[u]);
        }
        for (; r < a.rows; r += kWaves) twosum_add(s, c, base[size_t(r) * a.rstride]);
        ws_s[wave][col] = s;
        ws_c[wave][col] = c;
    }
    __syncthreads();
    if (wave != 0) {
        if (!end || !refine || wave_refine) return;
    } else {
        double mine = 0.0;  // the value of column `lane` (first pass)
        for (int col = lane; col < ncol; col += 64) {
            double s = ws_s[0][col], c = ws_c[0][col];
            for (int w = 1; w < kWaves; ++w) {
                twosum_add(s, c, ws_s[w][col]);
                c += ws_c[w][col];
            }
            const double val = s + c;
            double hi, lo;
            if (a.flags & MERGE_BEGIN) {
                hi = val;
                lo = 0.0;
            } else {  // double-double accumulation across chunks
                hi = a.acc[off + col];
                lo = a.acc[a.pstride + off + col];
                const double t = hi + val;
                const double bp = t - hi;
                lo += (hi - (t - bp)) + (val - bp);
                hi = t;
            }
            if (a.acc) {
                a.acc[off + col] = hi;
                a.acc[a.pstride + off + col] = lo;
            }
            if (end) {
                const double v = hi + lo;
                a.last[off + col] = v;
                fin[col] = v;
                if (col == lane) mine = v;
            }
        }
        if (!end) return;
        if (g == 0) {
            const double S2 = __shfl(mine, 1, 64);
            if (lane == 0) finish_iteration(a, mine, S2);
            return;
        }
        if (wave_refine) {
            refine_dim_wave(a, g - 1, mine, Eb, Eb1);
            return;
        }
        if (!refine) return;
    }
    // N > 64: the whole block refines from fin (LDS)
    __syncthreads();
    refine_dim(a, g - 1, fin, Eo);
}

// Inverse-variance combination of the recorded iterations flagged for it
// ("value +- error", Table 1): I = sum(I_t/var_t)/sum(1/var_t),
// sigma = sum(1/var_t)^(-1/2), chi^2/dof = sum (I_t - I)^2/var_t / (m - 1).
// Sums run in record order, as the method states them (one thread).
__device__ static void combine_records(const double* records, const int32_t* rec_flag, int n_rec, DevResult* R)
{
    double sw = 0.0, swi = 0.0;
    int m = 0;
    for (int k = 0; k < n_rec; ++k) {
        if (rec_flag[k]) {
            sw = sw + 1.0 / records[2 * k + 1];
            swi = swi + records[2 * k] / records[2 * k + 1];
            ++m;
        }
    }
    const double mean = swi / sw;
    double chi2 = 0.0;
    for (int k = 0; k < n_rec; ++k) {
        if (rec_flag[k]) {
            const double u = records[2 * k] - mean;
            chi2 = chi2 + u * u / records[2 * k + 1];
        }
    }
    const double nan = __builtin_nan("");
    R->integral = m > 0 ? mean : nan;
    R->sigma = m > 0 ? sqrt(1.0 / sw) : nan;
    R->chi2_dof = m > 1 ? chi2 / double(m - 1) : nan;
    R->n_combined = m;
}

}  // namespace vegas
