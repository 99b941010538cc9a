// Reduction, statistics and refinement kernels of one Vegas iteration.
//
// k_merge sums the per-block partial rows (S1, S2, H[d][N]) of the event
// kernel into one row, in a fixed order, with one block per column group:
// group 0 holds S1 and S2, group 1+i the N histogram bins of dimension i.
// Each block folds its sums into the iteration's double-double accumulator
// (several chunks form one iteration) and, at the end of the iteration,
// either records the statistics (group 0) or refines its dimension of the
// grid (groups 1..d, when asked).  No block waits for another and no
// device-wide fence is needed: the next kernel on the stream sees the result.
#include "grid_ops.hpp"

namespace vegas {

__global__ __launch_bounds__(kMergeThreads) void k_merge(MergeArgs a)
{
    if (int(blockIdx.x) == a.d + 1) {  // MERGE_GRAD: the gradient rows, scaled by 1/M
        adjoint_merge_block(a.gpart, a.rows, a.d, 1.0 / a.M, a.grad_out, 0);
        return;
    }
    merge_group(a, blockIdx.x);
}

// grad = gout * G, rounded once to the output's precision.
__global__ void k_grad_scale(const double* G, const double* gout, void* grad, int n, int grad_fp32)
{
    const double s = *gout;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double g = s * G[j];
        if (grad_fp32)
            static_cast<float*>(grad)[j] = float(g);
        else
            static_cast<double*>(grad)[j] = g;
    }
}

// Stand-alone refinement from the stored histograms of the last iteration.
__global__ __launch_bounds__(kMergeThreads) void k_refine(MergeArgs a)
{
    __shared__ double h[kMaxBins], Eo[kMaxBins + 1];
    const int i = blockIdx.x;
    for (int b = threadIdx.x; b < a.N; b += blockDim.x) h[b] = a.last[2 + size_t(i) * a.N + b];
    for (int b = threadIdx.x; b <= a.N; b += blockDim.x) Eo[b] = a.edges[size_t(i) * (a.N + 1) + b];
    __syncthreads();
    refine_any(a, i, h, Eo);
}

// Derived constants of the integrand (see DevConst), by one thread.
__device__ static void prepare_consts(int prec, int kind, int d, int N, const double* __restrict__ q,
                                      DevConst* __restrict__ c)
{
    const double pi = 3.14159265358979323846;
    const double log2e = 1.4426950408889634074;
    c->n_bins = N;
    c->pad1 = 0;
    c->two_m32 = 0x1p-32;
    c->dscale32 = width_scale32(N);
    const int ws = int(rint(log2(double(N))));
    double nd = 1.0;
    for (int i = 0; i < d; ++i) nd = nd * double(N);
    c->Cw = prec == FP64 ? nd : ldexp(nd, -ws * d);
    double Cf = 0.0;
    c->kexp64 = c->kexp2_64 = c->inv_a = 0.0;
    c->kexp32 = c->ka32 = c->pad0 = 0.0f;
    for (int i = 0; i < kMaxDim; ++i) {
        c->p1_64[i] = c->p2_64[i] = c->cA64[i] = c->cB64[i] = 0.0;
        c->p1_32[i] = c->p2_32[i] = 0.0f;
    }
    for (int i = 0; i < d; ++i) table_centres(kind, d, i, q, c->cA64[i], c->cB64[i]);
    if (kind == GAUSS || kind == BIMODAL) {
        const double a = q[0];
        Cf = pow(a * sqrt(pi), double(-d));
        if (kind == BIMODAL) Cf = 0.5 * Cf;
        c->kexp64 = 1.0 / (a * a);
        c->kexp2_64 = log2e / (a * a);
        c->inv_a = 1.0 / a;
        c->kexp32 = float(log2e / (a * a));
        c->ka32 = float(1.0 / (a * a));
        for (int i = 0; i < d; ++i) {
            c->p1_64[i] = q[1 + i];
            if (kind == BIMODAL) c->p2_64[i] = q[1 + d + i] - q[1 + i];  // FP64 map: u_B = u_A - (muB - muA)
        }
    } else if (kind == GENZ_DISC) {
        // nu exp(sum c x) = [nu e^{sum c a}] exp(sum c (x - a)); per dimension
        // nu e^{c a} = c / (e^{c (1 - a)} - 1)
        Cf = 1.0;
        c->kexp2_64 = log2e;
        for (int i = 0; i < d; ++i) {
            const double cc = q[i], aa = q[d + i];
            Cf = Cf * (cc / expm1(cc * (1.0 - aa)));
            c->p1_64[i] = cc;
            c->p2_64[i] = aa;
        }
    } else if (kind == USER) {
        // the caller's f carries its own normalisation; C = N^d
        Cf = 1.0;
    } else {
        // nu prod 1/(c^-2 + u^2) = [nu prod c^2] prod 1/(1 + c^2 u^2)
        Cf = 1.0;
        for (int i = 0; i < d; ++i) {
            const double cc = q[i], aa = q[d + i];
            Cf = Cf * (cc / (atan(cc * (1.0 - aa)) + atan(cc * aa)));
            c->p1_64[i] = cc * cc;
            c->p2_64[i] = aa;
            c->p1_32[i] = float(cc * cc);
        }
    }
    c->Cf = Cf;
    c->C = Cf * c->Cw;
}

__global__ void k_prepare(int prec, int kind, int d, int N, const double* __restrict__ q,
                          DevConst* __restrict__ c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) prepare_consts(prec, kind, d, N, q, c);
}

// New integrand parameters in one launch (block i: dimension i): every block
// reads the caller's n values (FP64, or FP32 widened exactly), block 0 stores
// them and the derived constants, and each block rebuilds its dimension's
// tables (whose FP32 entries are offsets from the parameters' centres) with
// the centres taken from the parameters themselves, so no block waits for
// another.
__global__ __launch_bounds__(256) void k_set_params(int prec, int kind, int d, int N, const void* __restrict__ src,
                                                    const void* __restrict__ rest, int n, int is_fp32, ProblemPtrs p)
{
    __shared__ double q[kMaxParams];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        // value k: src[k], or with rest given, src[0] and rest[k - 1]
        const void* a = rest && k > 0 ? rest : src;
        const int j = rest && k > 0 ? k - 1 : k;
        q[k] = is_fp32 ? double(static_cast<const float*>(a)[j]) : static_cast<const double*>(a)[j];
    }
    __syncthreads();
    const int i = blockIdx.x;
    if (i == 0) {
        for (int k = threadIdx.x; k < n; k += blockDim.x) p.params[k] = q[k];
        if (threadIdx.x == 0) prepare_consts(prec, kind, d, N, q, p.cst);
    }
    double cA, cB;
    table_centres(kind, d, i, q, cA, cB);
    const float ds = width_scale32(N);
    const double* E = p.edges + size_t(i) * (N + 1);
    for (int b = threadIdx.x; b < N; b += blockDim.x)
        write_table_entry(i, b, E[b], E[b + 1], cA, cB, ds, kind, N, p.tab64, p.tab32);
    if (kind == GENZ_DISC && threadIdx.x == 0) p.thr[i] = disc_threshold(E, N, cA);
}

// Uniform grid E_k = k/N and a clean state (tables: k_build_tables).
__global__ void k_init_state(ProblemPtrs p, int d, int N, int pstride)
{
    const int i = blockIdx.x;
    if (i < d) {
        double* E = p.edges + size_t(i) * (N + 1);
        for (int k = threadIdx.x; k <= N; k += blockDim.x) E[k] = double(k) / double(N);
        return;
    }
    for (int k = threadIdx.x; k < 2 * pstride; k += blockDim.x) p.acc[k] = 0.0;
    for (int k = threadIdx.x; k < pstride; k += blockDim.x) p.last[k] = 0.0;
    for (int k = threadIdx.x; k < kHistSlots * (pstride - 2); k += blockDim.x) p.hslots[k] = 0.0;
    for (int k = threadIdx.x; k < 2 * kMaxRecords; k += blockDim.x) p.records[k] = 0.0;
    for (int k = threadIdx.x; k < kMaxRecords; k += blockDim.x) p.rec_flag[k] = 0;
    if (threadIdx.x == 0) {
        const double nan = __builtin_nan("");
        DevResult* R = p.result;
        R->integral = R->sigma = R->chi2_dof = R->last_integral = R->last_var = nan;
        R->n_iter = R->n_combined = R->n_events = R->n_nonfinite = 0;
    }
}

__global__ void k_zero(double* x, size_t n)
{
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x)
        x[k] = 0.0;
}

__global__ void k_build_tables(ProblemPtrs p, int kind, int N)
{
    const int i = blockIdx.x;
    write_tables(i, p.edges + size_t(i) * (N + 1), p.cst, kind, N, p.tab64, p.tab32, p.thr);
}

__global__ void k_combine(const double* records, const int32_t* rec_flag, int n_rec, DevResult* R)
{
    if (threadIdx.x == 0) combine_records(records, rec_flag, n_rec, R);
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
    const int blocks = a.d + 1 + ((a.flags & MERGE_GRAD) ? 1 : 0);
    hipLaunchKernelGGL(k_merge, dim3(blocks), dim3(kMergeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_grad_scale(const double* G, const double* gout, void* grad, int n, int grad_fp32, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_scale, dim3(1), dim3(128), 0, s, G, gout, grad, n, grad_fp32);
    return hipGetLastError();
}

hipError_t launch_refine(const MergeArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_refine, dim3(a.d), dim3(kMergeThreads), 0, s, a);
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

hipError_t launch_zero(double* x, size_t n, hipStream_t s)
{
    const unsigned blocks = unsigned(n / 256 + 1 < 1024 ? n / 256 + 1 : 1024);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_build_tables(const ProblemPtrs& p, int kind, int d, int N, hipStream_t s)
{
    hipLaunchKernelGGL(k_build_tables, dim3(d), dim3(256), 0, s, p, kind, N);
    return hipGetLastError();
}

hipError_t launch_combine(const double* records, const int32_t* rec_flag, int n_rec, DevResult* result,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(64), 0, s, records, rec_flag, n_rec, result);
    return hipGetLastError();
}

hipError_t launch_set_params(int prec, int kind, int d, int N, const void* src, int n, int is_fp32,
                             const ProblemPtrs& p, hipStream_t s, const void* rest)
{
    hipLaunchKernelGGL(k_set_params, dim3(d), dim3(256), 0, s, prec, kind, d, N, src, rest, n, is_fp32, p);
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
