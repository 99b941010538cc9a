// vegas_init_grid_noalloc: a context whose device workspace is a static
// array of this library, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).  The array is
// `scratch` below; each device holds its own copy, whose device address host
// code takes from hipGetSymbolAddress once per device (the array's name in
// host code is only a host-side stand-in, never a device address).
#include <mutex>

#include "capi_util.hpp"
#include "vegas_internal.hpp"

using namespace vegas;

// Every admissible (dim, n_bins) fits: a single-problem workspace (grid,
// tables, histogram slots, accumulators, records, adjoint partials) is about
// 1.2 MiB plus 128 bytes per (dimension, bin), and the event kernel's LDS
// limit keeps dim * n_bins near 10^4 at most (2.32 MiB, FP32 d = 48, N = 213).
constexpr size_t kScratchBytes = size_t(4) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch_ptr[kStaticDevices] = {};  // device address of `scratch`, per device

}  // namespace

extern "C" vegas_status vegas_init_grid_noalloc(vegas_ctx** out, const vegas_desc* desc, vegas_stream_t stream)
{
    if (!out) return fail(VEGAS_EINVAL, "out is NULL");
    *out = nullptr;
    vegas_status st = check_desc(desc);
    if (st != VEGAS_OK) return st;
    if (desc->integrand == VEGAS_USER)
        return fail(VEGAS_EUNSUPPORTED, "user integrands are compiled and loaded at init: use vegas_init_user");
    const size_t need = make_layout(desc->dim, desc->n_bins).total;
    if (need > kScratchBytes)
        return fail(VEGAS_EUNSUPPORTED, "dim %d, n_bins %d need %zu bytes of workspace; the static one holds %zu",
                    desc->dim, desc->n_bins, need, kScratchBytes);
    int dev = 0;
    VEGAS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticDevices)
        return fail(VEGAS_EUNSUPPORTED, "device %d: static workspaces cover devices 0..%d", dev, kStaticDevices - 1);
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            const hipError_t he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (he != hipSuccess || !p)
                return fail(VEGAS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(he));
            g_scratch_ptr[dev] = p;
        }
        ws = g_scratch_ptr[dev];
    }
    return init_static_ctx(out, desc, dev, ws, kScratchBytes, stream);
}
