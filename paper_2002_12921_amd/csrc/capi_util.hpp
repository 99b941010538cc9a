// Host-side helpers shared by the single-problem and batch entry points.
#pragma once

#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "vegas.h"

namespace vegas {

extern thread_local std::string g_err;

// Records a formatted message for vegas_last_error() and returns st.
vegas_status fail(vegas_status st, const char* fmt, ...);

// Number of integrand parameters of a kind at dimension d (-1: unknown kind).
int expected_params(int kind, int d);

// Full validation of a problem description (no HIP call).
vegas_status check_desc(const vegas_desc* d);

// Devices that can hold a static (allocation-free) context.
constexpr int kStaticDevices = 16;

// The device's static context of vegas_init_grid_noalloc, (re)initialised
// over the static device workspace ws (ws_bytes); allocates nothing.
vegas_status init_static_ctx(vegas_ctx** out, const vegas_desc* desc, int device, void* ws, size_t ws_bytes,
                             vegas_stream_t stream);

// A roctx range around one entry point's launches: rocprofv3 --marker-trace
// shows each iteration, refinement and batch step as a named range.  Without
// a profiler attached a push or pop is a call through an empty dispatch table.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

}  // namespace vegas

#define VEGAS_HIP(expr)                                                                               \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return vegas::fail(VEGAS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
