// Reduction, statistics and refinement kernels of one Vegas iteration.
//
// k_merge sums the per-block partial rows (S1, S2, H[d][N]) into one row in a
// fixed order: a grid of (1 + d) column groups x `splits` row ranges; group 0
// holds S1 and S2, group 1+i the N histogram bins of dimension i.  Each block
// writes a level-2 row; the last block of each group (atomic ticket) adds the
// level-2 rows in order (Neumaier), folds the result into the iteration's
// double-double accumulator (several chunks form one iteration) and, at the
// end of the iteration, either records the statistics (group 0) or refines
// its dimension of the grid (groups 1..d, when asked).  Tickets are reset by
// the last block, so the kernel can be replayed without host work.
#include "device_common.hpp"

namespace vegas {

// Statistics of one iteration and the running combination ("value +- error",
// Table 1; inverse-variance weighting of Lepage 1978 sec. 3).
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

    double sw = 0.0, swi = 0.0;
    int m = 0;
    for (int k = 0; k <= rec; ++k) {
        if (a.rec_flag[k]) {
            sw = sw + 1.0 / a.records[2 * k + 1];
            swi = swi + a.records[2 * k] / a.records[2 * k + 1];
            ++m;
        }
    }
    const double mean = swi / sw;
    double chi2 = 0.0;
    for (int k = 0; k <= rec; ++k) {
        if (a.rec_flag[k]) {
            const double u = a.records[2 * k] - mean;
            chi2 = chi2 + u * u / a.records[2 * k + 1];
        }
    }
    const double nan = __builtin_nan("");
    R->integral = m > 0 ? mean : nan;
    R->sigma = m > 0 ? sqrt(1.0 / sw) : nan;
    R->chi2_dof = m > 1 ? chi2 / double(m - 1) : nan;
    R->n_combined = m;
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
// The two running sums are taken in bin order by one thread, as the method
// states them; each new edge is found by bisection on the cumulative sums.
__device__ static void refine_dim(const MergeArgs& a, int i, const double* h)
{
    const int N = a.N;
    __shared__ double Eo[kMaxBins + 1], En[kMaxBins + 1], s_[kMaxBins], r_[kMaxBins],
        A_[kMaxBins + 1];
    __shared__ double ssum_s;
    __shared__ int skip;
    double* E = a.edges + size_t(i) * (N + 1);
    for (int k = threadIdx.x; k <= N; k += blockDim.x) Eo[k] = E[k];
    for (int b = threadIdx.x; b < N; b += blockDim.x) {
        const double l = b > 0 ? h[b - 1] : 0.0;
        const double c = h[b];
        const double rgt = b < N - 1 ? h[b + 1] : 0.0;
        if (b == 0)
            s_[b] = (c + rgt) / 2.0;
        else if (b == N - 1)
            s_[b] = (l + c) / 2.0;
        else
            s_[b] = (l + c + rgt) / 3.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0, ss = 0.0;
        for (int b = 0; b < N; ++b) {
            tot = tot + h[b];
            ss = ss + s_[b];
        }
        skip = (tot == 0.0);
        ssum_s = ss;
    }
    __syncthreads();
    if (skip) return;  // empty histogram: the grid and its tables stay
    const double ssum = ssum_s;
    for (int b = threadIdx.x; b < N; b += blockDim.x) r_[b] = damp(s_[b] / ssum, a.alpha);
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        A_[0] = 0.0;
        for (int b = 0; b < N; ++b) {
            acc = acc + r_[b];
            A_[b + 1] = acc;  // damped weight in bins 0..b
        }
    }
    __syncthreads();
    const double R = A_[N];
    for (int k = threadIdx.x; k <= N; k += blockDim.x) {
        double e;
        if (k == 0 || k == N) {
            e = Eo[k];
        } else {
            const double level = double(k) * R / double(N);
            // first b with A[b+1] >= level (bins with r = 0 never qualify first)
            int lo = 0, hi = N - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (A_[mid + 1] >= level)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            const int b = lo;
            e = Eo[b] + (level - A_[b]) / r_[b] * (Eo[b + 1] - Eo[b]);
        }
        En[k] = e;
        E[k] = e;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < N; b += blockDim.x) {
        const double lo = En[b], w = En[b + 1] - En[b];
        a.tab64[size_t(i) * N + b] = make_double2(lo, w);
        a.tab32[size_t(i) * N + b] = make_float2(float(lo), float(w));
    }
}

__global__ __launch_bounds__(256) void k_merge(MergeArgs a)
{
    const int g = blockIdx.x;
    const int rs = blockIdx.y;
    const int ncol = g == 0 ? 2 : a.N;
    const int off = g == 0 ? 0 : 2 + (g - 1) * a.N;
    const int CW = ncol <= 64 ? 64 : (ncol <= 128 ? 128 : 256);
    const int RL = 256 / CW;
    const int col = threadIdx.x % CW, rl = threadIdx.x / CW;
    const int r0 = int(int64_t(rs) * a.rows / a.splits);
    const int r1 = int(int64_t(rs + 1) * a.rows / a.splits);

    __shared__ double ps[256], pc[256], fin[kMaxBins + 1];
    __shared__ int is_last;
    double s = 0.0, c = 0.0;
    if (col < ncol)
        for (int r = r0 + rl; r < r1; r += RL) neumaier_add(s, c, a.partials[size_t(r) * a.pstride + off + col]);
    ps[threadIdx.x] = s;
    pc[threadIdx.x] = c;
    __syncthreads();
    if (rl == 0 && col < ncol) {
        double S = 0.0, C = 0.0;
        for (int k = 0; k < RL; ++k) {
            neumaier_add(S, C, ps[k * CW + col]);
            C += pc[k * CW + col];
        }
        a.level2[size_t(rs) * a.pstride + off + col] = S + C;
    }

    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = (atomicAdd(&a.tickets[g], 1u) == unsigned(a.splits - 1));
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    if (threadIdx.x == 0) a.tickets[g] = 0u;

    for (int k = threadIdx.x; k < ncol; k += blockDim.x) {
        double S = 0.0, C = 0.0;
        for (int r = 0; r < a.splits; ++r) neumaier_add(S, C, a.level2[size_t(r) * a.pstride + off + k]);
        const double val = S + C;
        double hi, lo;
        if (a.flags & MERGE_BEGIN) {
            hi = val;
            lo = 0.0;
        } else {  // double-double accumulation across chunks
            hi = a.acc[off + k];
            lo = a.acc[a.pstride + off + k];
            const double t = hi + val;
            const double bp = t - hi;
            lo += (hi - (t - bp)) + (val - bp);
            hi = t;
        }
        a.acc[off + k] = hi;
        a.acc[a.pstride + off + k] = lo;
        if (a.flags & MERGE_END) {
            const double v = hi + lo;
            a.last[off + k] = v;
            fin[k] = v;
        }
    }
    if (!(a.flags & MERGE_END)) return;
    __syncthreads();
    if (g == 0) {
        if (threadIdx.x == 0) finish_iteration(a, fin[0], fin[1]);
    } else if (a.flags & MERGE_REFINE) {
        refine_dim(a, g - 1, fin);
    }
}

// Stand-alone refinement from the stored histograms of the last iteration.
__global__ __launch_bounds__(256) void k_refine(MergeArgs a)
{
    __shared__ double h[kMaxBins];
    const int i = blockIdx.x;
    for (int b = threadIdx.x; b < a.N; b += blockDim.x) h[b] = a.last[2 + size_t(i) * a.N + b];
    __syncthreads();
    refine_dim(a, i, h);
}

// Derived constants of the integrand (see DevConst).
__global__ void k_prepare(int prec, int kind, int d, int N, const double* __restrict__ q,
                          DevConst* __restrict__ c)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double pi = 3.14159265358979323846;
    const double log2e = 1.4426950408889634074;
    c->nscale = double(N) / 4294967296.0;
    c->nhalf = double(N) / 8589934592.0;
    // FP32 width product: multiply by 2^wshift per dimension, wshift = round(log2 N)
    const int wshift = int(rint(log2(double(N))));
    c->wgroup32 = ldexpf(1.0f, 4 * wshift);
    c->wlast32 = ldexpf(1.0f, (d % 4) * wshift);
    double nd = 1.0;
    for (int i = 0; i < d; ++i) nd = nd * double(N);
    c->Cw = prec == FP64 ? nd : ldexp(nd, -wshift * d);
    double Cf = 0.0;
    c->kexp64 = c->inv_a = 0.0;
    c->kexp32 = c->ka32 = 0.0f;
    for (int i = 0; i < kMaxDim; ++i) {
        c->p1_64[i] = c->p2_64[i] = 0.0;
        c->p1_32[i] = c->p2_32[i] = 0.0f;
    }
    if (kind == GAUSS || kind == BIMODAL) {
        const double a = q[0];
        Cf = pow(a * sqrt(pi), double(-d));
        if (kind == BIMODAL) Cf = 0.5 * Cf;
        c->kexp64 = 1.0 / (a * a);
        c->inv_a = 1.0 / a;
        c->kexp32 = float(log2e / (a * a));
        c->ka32 = float(1.0 / (a * a));
        for (int i = 0; i < d; ++i) {
            c->p1_64[i] = q[1 + i];
            c->p1_32[i] = float(q[1 + i]);
            if (kind == BIMODAL) {
                c->p2_64[i] = q[1 + d + i];
                c->p2_32[i] = float(q[1 + d + i]);
            }
        }
    } else if (kind == GENZ_DISC) {
        // nu exp(sum c x) = [nu e^{sum c}] exp(sum c (x - 1)); nu e^{c} per dim = c/(1 - e^{c(a-1)})
        Cf = 1.0;
        for (int i = 0; i < d; ++i) {
            const double cc = q[i], aa = q[d + i];
            Cf = Cf * (cc / (1.0 - exp(cc * (aa - 1.0))));
            c->p1_64[i] = cc;
            c->p2_64[i] = aa;
            c->p1_32[i] = float(cc * log2e);
            c->p2_32[i] = float(aa);
        }
    } else {
        // nu prod 1/(c^-2 + u^2) = [nu prod c^2] prod 1/(1 + c^2 u^2)
        Cf = 1.0;
        for (int i = 0; i < d; ++i) {
            const double cc = q[i], aa = q[d + i];
            Cf = Cf * (cc / (atan(cc * (1.0 - aa)) + atan(cc * aa)));
            c->p1_64[i] = cc * cc;
            c->p2_64[i] = aa;
            c->p1_32[i] = float(cc * cc);
            c->p2_32[i] = float(aa);
        }
    }
    c->Cf = Cf;
    c->C = Cf * c->Cw;
}

// Uniform grid E_k = k/N, its tables, and a clean state.
__global__ void k_init_state(ProblemPtrs p, int d, int N, int pstride)
{
    const int i = blockIdx.x;
    if (i < d) {
        double* E = p.edges + size_t(i) * (N + 1);
        for (int k = threadIdx.x; k <= N; k += blockDim.x) E[k] = double(k) / double(N);
        for (int b = threadIdx.x; b < N; b += blockDim.x) {
            const double lo = double(b) / double(N), hi = double(b + 1) / double(N);
            p.tab64[size_t(i) * N + b] = make_double2(lo, hi - lo);
            p.tab32[size_t(i) * N + b] = make_float2(float(lo), float(hi - lo));
        }
        return;
    }
    for (int k = threadIdx.x; k < 2 * pstride; k += blockDim.x) p.acc[k] = 0.0;
    for (int k = threadIdx.x; k < pstride; k += blockDim.x) p.last[k] = 0.0;
    for (int k = threadIdx.x; k < 2 * kMaxRecords; k += blockDim.x) p.records[k] = 0.0;
    for (int k = threadIdx.x; k < kMaxRecords; k += blockDim.x) p.rec_flag[k] = 0;
    for (int k = threadIdx.x; k < kMaxDim + 8; k += blockDim.x) p.tickets[k] = 0u;
    if (threadIdx.x == 0) {
        const double nan = __builtin_nan("");
        DevResult* R = p.result;
        R->integral = R->sigma = R->chi2_dof = R->last_integral = R->last_var = nan;
        R->n_iter = R->n_combined = R->n_events = R->n_nonfinite = 0;
    }
}

__global__ void k_build_tables(double* edges, double2* tab64, float2* tab32, int N)
{
    const int i = blockIdx.x;
    const double* E = edges + size_t(i) * (N + 1);
    for (int b = threadIdx.x; b < N; b += blockDim.x) {
        const double lo = E[b], w = E[b + 1] - E[b];
        tab64[size_t(i) * N + b] = make_double2(lo, w);
        tab32[size_t(i) * N + b] = make_float2(float(lo), float(w));
    }
}

__global__ void k_params_from(const void* src, int n, int is_fp32, double* dst)
{
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        dst[k] = is_fp32 ? double(static_cast<const float*>(src)[k]) : static_cast<const double*>(src)[k];
}

__global__ void k_reset_results(double* records, int32_t* rec_flag, DevResult* R)
{
    for (int k = threadIdx.x; k < 2 * kMaxRecords; k += blockDim.x) records[k] = 0.0;
    for (int k = threadIdx.x; k < kMaxRecords; k += blockDim.x) rec_flag[k] = 0;
    if (threadIdx.x == 0) {
        const double nan = __builtin_nan("");
        R->integral = R->sigma = R->chi2_dof = R->last_integral = R->last_var = nan;
        R->n_iter = R->n_combined = R->n_events = R->n_nonfinite = 0;
    }
}

__global__ void k_copy_last(const DevResult* R, double* out)
{
    if (threadIdx.x == 0) {
        out[0] = R->last_integral;
        out[1] = sqrt(R->last_var);
    }
}

// ---------------------------------------------------------------------------

hipError_t launch_merge(const MergeArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_merge, dim3(a.d + 1, a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_refine(const MergeArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_refine, dim3(a.d), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prepare(int prec, int kind, int d, int N, const double* params, DevConst* cst,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(64), 0, s, prec, kind, d, N, params, cst);
    return hipGetLastError();
}

hipError_t launch_init_state(const ProblemPtrs& p, int d, int N, int pstride, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(d + 1), dim3(256), 0, s, p, d, N, pstride);
    return hipGetLastError();
}

hipError_t launch_build_tables(double* edges, double2* tab64, float2* tab32, int d, int N,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_build_tables, dim3(d), dim3(256), 0, s, edges, tab64, tab32, N);
    return hipGetLastError();
}

hipError_t launch_params_from(const void* src, int n, int is_fp32, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_params_from, dim3(1), dim3(256), 0, s, src, n, is_fp32, dst);
    return hipGetLastError();
}

hipError_t launch_reset_results(double* records, int32_t* rec_flag, DevResult* result,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_results, dim3(1), dim3(256), 0, s, records, rec_flag, result);
    return hipGetLastError();
}

hipError_t launch_copy_last(const DevResult* result, double* out2, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_last, dim3(1), dim3(64), 0, s, result, out2);
    return hipGetLastError();
}

}  // namespace vegas
