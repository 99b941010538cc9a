// Device routines shared by the single-problem and batched reduction kernels:
// the statistics of one iteration, the grid tables and the refinement.
#pragma once

#include "device_common.hpp"

namespace vegas {

// Statistics of one iteration (Lepage 1978 sec. 3): I_t = S1/M and the
// variance of that mean, var_t = (S2/M - I_t^2)/(M - 1).  The iteration is
// recorded; the combination over recorded iterations runs in k_combine.
__device__ static void finish_iteration(const MergeArgs& a, double S1, double S2)
{
    const double M = a.M;
    const double I = S1 / M;
    const double var = (S2 / M - I * I) / (M - 1.0);
    const bool ok = isfinite(I) && isfinite(var);
    const int rec = a.rec_idx;
    a.records[2 * rec] = I;
    a.records[2 * rec + 1] = var;
    a.rec_flag[rec] = (ok && !(a.flags & MERGE_NO_COMBINE)) ? 1 : 0;
    DevResult* R = a.result;
    R->last_integral = I;
    R->last_var = var;
    R->n_iter = rec + 1;
    R->n_events += int64_t(M);
    if (!ok) R->n_nonfinite += 1;
}

// Grid tables of dimension i from its edges E[0..N] (any address space).
//   FP64: (E_b, E_{b+1} - E_b)
//   FP32: with W = RN32(E_{b+1} - E_b), S = 2^(ws + 32) and g = E_b + h W / 2^32
//         (h = 1/2 for odd N, else 0),
//         (RN32((g - cA) S), [RN32((g - cB) S),] W 2^ws)
//   The event kernel forms (x - c) S = RN32(lo) W 2^ws + first entry.
__device__ static void write_tables(int i, const double* E, const DevConst* __restrict__ c, int kind,
                                    int N, double2* tab64, float* tab32)
{
    const double cA = c->cA64[i], cB = c->cB64[i];
    const double sw = 1.0 / double(c->dscale32);  // 2^ws
    const double S = sw * 0x1p32;
    const double h = (N & 1) ? 0x1p-33 : 0.0;     // h / 2^32
    for (int b = threadIdx.x; b < N; b += blockDim.x) {
        const double lo = E[b], w = E[b + 1] - E[b];
        tab64[size_t(i) * N + b] = make_double2(lo, w);
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
}

// Damping of the refinement: r(s) = ((s - 1)/ln s)^alpha, r(0) = 0, r(1) = 1.
__device__ static double damp(double s, double alpha)
{
    if (s == 0.0) return 0.0;
    if (s == 1.0) return 1.0;
    return pow((s - 1.0) / log(s), alpha);
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
    if (tot[0] == 0.0) return;  // empty histogram: the grid and its tables stay
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
    write_tables(i, En, a.cst, a.kind, N, a.tab64, a.tab32);
}

// One column group of the reduction (group 0: S1, S2; group 1+i: the
// histogram of dimension i): the partial rows are summed in order, folded
// into the chunk accumulator (when there is one), and at the end of the
// iteration the group records the statistics or refines its dimension.
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
    int CW = 2;
    while (CW < ncol) CW <<= 1;          // columns per row pass (power of two)
    const int RL = kMergeThreads / CW;   // row lanes
    const int col = threadIdx.x % CW, rl = threadIdx.x / CW;

    __shared__ double ps[kMergeThreads], pc[kMergeThreads], fin[kMaxBins + 1], Eo[kMaxBins + 1];
    const bool refine = (a.flags & MERGE_END) && (a.flags & MERGE_REFINE) && g > 0;
    // the edges the refinement needs, fetched while the rows are summed
    if (refine && int(threadIdx.x) <= a.N) Eo[threadIdx.x] = a.edges[size_t(g - 1) * (a.N + 1) + threadIdx.x];
    double s = 0.0, c = 0.0;
    if (col < ncol) {
        // rows rl, rl + RL, ...: loads issued sixteen at a time, then added in order
        const double* base = a.partials + off + col;
        int r = rl;
        for (; r + 15 * RL < a.rows; r += 16 * RL) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = base[size_t(r + u * RL) * a.pstride];
#pragma unroll
            for (int u = 0; u < 16; ++u) twosum_add(s, c, v[u]);
        }
        if (r + 7 * RL < a.rows) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = base[size_t(r + u * RL) * a.pstride];
#pragma unroll
            for (int u = 0; u < 8; ++u) twosum_add(s, c, v[u]);
            r += 8 * RL;
        }
        for (; r < a.rows; r += RL) twosum_add(s, c, base[size_t(r) * a.pstride]);
    }
    ps[threadIdx.x] = s;
    pc[threadIdx.x] = c;
    __syncthreads();
    // combine the row lanes in a fixed order (tree over lanes)
    for (int half = RL / 2; half > 0; half >>= 1) {
        if (rl < half) {
            const int o = threadIdx.x + half * CW;
            double S = ps[threadIdx.x], C = pc[threadIdx.x];
            twosum_add(S, C, ps[o]);
            ps[threadIdx.x] = S;
            pc[threadIdx.x] = C + pc[o];
        }
        __syncthreads();
    }
    if (rl == 0 && col < ncol) {
        const double val = ps[col] + pc[col];
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
        if (a.flags & MERGE_END) {
            const double v = hi + lo;
            a.last[off + col] = v;
            fin[col] = v;
        }
    }
    if (!(a.flags & MERGE_END)) return;
    __syncthreads();
    if (g == 0) {
        if (threadIdx.x == 0) finish_iteration(a, fin[0], fin[1]);
    } else if (refine) {
        refine_dim(a, g - 1, fin, Eo);
    }
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
