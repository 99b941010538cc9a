// Issue-rate probes of the VALU instruction classes the event kernel's
// roofline weighs (vegas_probe_issue_rates): a 32x32->64 multiply-add
// (v_mad_u64_u32) beside a three-way XOR (v_bitop3_b32), the XOR alone, the
// FP32 fma and the FP32 base-2 exponential (a transcendental).  Each thread
// runs eight independent chains, so that issue and not latency sets the pace,
// and the grid keeps eight waves on every SIMD.  The host turns kernel times
// into VALU instructions per second over the chip, with the instructions per
// chain step that each loop body compiles to.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "capi_util.hpp"
#include "vegas_internal.hpp"

using namespace vegas;

namespace {

constexpr int kChains = 8;
constexpr int kProbeThreads = 256;
constexpr int kProbeWavesPerSimd = 8;

__device__ __forceinline__ uint32_t xor3p(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// per chain step: p = a * M (64-bit product), a = hi(p) ^ b ^ k, b = lo(p)
__global__ __launch_bounds__(kProbeThreads) void k_probe_mad(uint32_t* out, int n, uint32_t k)
{
    uint32_t a[kChains], b[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = threadIdx.x * 2654435761u + uint32_t(c);
        b[c] = blockIdx.x * 40503u + uint32_t(c) * 7u;
    }
    for (int it = 0; it < n; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const uint64_t p = uint64_t(a[c]) * 0xD2511F53u;
            a[c] = xor3p(uint32_t(p >> 32), b[c], k);
            b[c] = uint32_t(p);
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= a[c] ^ b[c];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = r;
}

// per chain step: a = a ^ b ^ k, b = b ^ a ^ (k + 1)
__global__ __launch_bounds__(kProbeThreads) void k_probe_xor(uint32_t* out, int n, uint32_t k)
{
    uint32_t a[kChains], b[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = threadIdx.x * 2654435761u + uint32_t(c);
        b[c] = blockIdx.x * 40503u + uint32_t(c) * 7u;
    }
    for (int it = 0; it < n; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            a[c] = xor3p(a[c], b[c], k);
            b[c] = xor3p(b[c], a[c], k + 1u);
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= a[c] ^ b[c];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = r;
}

// per chain step: x = fma(x, s, 1/4)
__global__ __launch_bounds__(kProbeThreads) void k_probe_fma(uint32_t* out, int n, float s)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = float(threadIdx.x) * 1e-3f + float(c);
    for (int it = 0; it < n; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], s, 0.25f);
    }
    float r = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r += x[c];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = __float_as_uint(r);
}

// per chain step: x = 2^-x (x stays in (0, 1])
__global__ __launch_bounds__(kProbeThreads) void k_probe_exp(uint32_t* out, int n, float s)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = float(threadIdx.x) * 1e-4f * s + float(c) * 0.1f;
    for (int it = 0; it < n; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
    }
    float r = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r += x[c];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = __float_as_uint(r);
}

}  // namespace

extern "C" vegas_status vegas_probe_issue_rates(void* dev_scratch, size_t bytes, int32_t iters, double* host_ms,
                                                int32_t* host_blocks, vegas_stream_t stream)
{
    if (!dev_scratch || !host_ms || !host_blocks) return fail(VEGAS_EINVAL, "NULL argument");
    if (iters < 1 || iters > (1 << 20)) return fail(VEGAS_EINVAL, "iters must be in [1, 2^20]");
    int dev = 0, cus = 0;
    VEGAS_HIP(hipGetDevice(&dev));
    VEGAS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // eight waves on each of a CU's four SIMDs, 4-wave blocks
    const int blocks = cus * 4 * kProbeWavesPerSimd / (kProbeThreads / 64);
    const size_t need = sizeof(uint32_t) * size_t(blocks) * kProbeThreads;
    if (bytes < need) return fail(VEGAS_EWORKSPACE, "probe scratch has %zu bytes, needs %zu", bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t* out = static_cast<uint32_t*>(dev_scratch);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    VEGAS_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    for (int which = 0; which < 4 && he == hipSuccess; ++which) {
        for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {  // the first launch warms up
            he = hipEventRecord(e0, s);
            if (he != hipSuccess) break;
            switch (which) {
            case 0: hipLaunchKernelGGL(k_probe_mad, dim3(blocks), dim3(kProbeThreads), 0, s, out, iters, 0x9E3779B9u); break;
            case 1: hipLaunchKernelGGL(k_probe_xor, dim3(blocks), dim3(kProbeThreads), 0, s, out, iters, 0x9E3779B9u); break;
            case 2: hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(kProbeThreads), 0, s, out, iters, 0.5f); break;
            default: hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(kProbeThreads), 0, s, out, iters, 1.0f); break;
            }
            he = hipGetLastError();
            if (he == hipSuccess) he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            host_ms[which] = double(ms);
        }
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (he != hipSuccess) return fail(VEGAS_EHIP, "probe: %s", hipGetErrorString(he));
    *host_blocks = blocks;
    return VEGAS_OK;
}
