// Runtime compilation of caller-supplied integrands with hipRTC.  The device
// headers of the library (vegas_internal.hpp, device_common.hpp) and the
// user-kernel template (k_user_rtc.hpp) are embedded as text at build time and
// handed to the runtime compiler as in-memory headers, so a user integrand runs
// on exactly the points, map and sums of the built-in kernels.
#include "rtc.hpp"

#include <hip/hiprtc.h>

#include <map>
#include <mutex>
#include <utility>

#include "capi_util.hpp"
#include "vegas_internal.hpp"
#include "vegas_rtc_sources.inc"  // kRtcInternal, kRtcCommon, kRtcUser (written by build.py)

namespace vegas {

namespace {

std::mutex g_cache_mu;
std::map<std::pair<int, std::string>, std::string> g_cache;  // key: (d + 1000 * prec, source)
constexpr size_t kCacheEntries = 64;

std::string program_log(hiprtcProgram p)
{
    size_t n = 0;
    if (hiprtcGetProgramLogSize(p, &n) != HIPRTC_SUCCESS || n == 0) return std::string();
    std::string log(n, '\0');
    if (hiprtcGetProgramLog(p, &log[0]) != HIPRTC_SUCCESS) return std::string();
    while (!log.empty() && log.back() == '\0') log.pop_back();
    return log;
}

}  // namespace

vegas_status rtc_compile(const char* source, int d, int prec, std::string& code, std::string& log)
{
    code.clear();
    log.clear();
    if (!source) return fail(VEGAS_EINVAL, "source is NULL");
    const bool fp32 = prec == FP32;
    const auto key = std::make_pair(d + (fp32 ? 1000 : 0), std::string(source));
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            code = it->second;
            return VEGAS_OK;
        }
    }
    // the caller's lines are numbered from 1 in file "integrand" in messages
    const std::string text = "#define VEGAS_DIM " + std::to_string(d) + "\n#define VEGAS_THREADS " +
                             std::to_string(kUserThreads) + (fp32 ? "\n#define VEGAS_FP32 1\ntypedef float vegas_real;"
                                                                  : "\ntypedef double vegas_real;") +
                             "\n#include \"device_common.hpp\"\n#line 1 \"integrand\"\n" + source +
                             "\n#include \"k_user_rtc.hpp\"\n";
    const char* headers[] = {kRtcInternal, kRtcCommon, kRtcUser};
    const char* names[] = {"vegas_internal.hpp", "device_common.hpp", "k_user_rtc.hpp"};
    hiprtcProgram prog = nullptr;
    hiprtcResult r = hiprtcCreateProgram(&prog, text.c_str(), "vegas_user.hip", 3, headers, names);
    if (r != HIPRTC_SUCCESS) return fail(VEGAS_EHIP, "hiprtcCreateProgram: %s", hiprtcGetErrorString(r));
    // no packed-FP32 instructions in generated code, as for the built-in kernels
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    r = hiprtcCompileProgram(prog, int(sizeof(opts) / sizeof(opts[0])), opts);
    log = program_log(prog);
    if (r != HIPRTC_SUCCESS) {
        (void)hiprtcDestroyProgram(&prog);
        return fail(VEGAS_ECOMPILE, "integrand source did not compile (%s): %.400s", hiprtcGetErrorString(r),
                    log.c_str());
    }
    size_t n = 0;
    r = hiprtcGetCodeSize(prog, &n);
    if (r == HIPRTC_SUCCESS) {
        code.resize(n);
        r = hiprtcGetCode(prog, &code[0]);
    }
    (void)hiprtcDestroyProgram(&prog);
    if (r != HIPRTC_SUCCESS || n == 0) {
        code.clear();
        return fail(VEGAS_EHIP, "hiprtcGetCode: %s", hiprtcGetErrorString(r));
    }
    std::lock_guard<std::mutex> g(g_cache_mu);
    if (g_cache.size() >= kCacheEntries) g_cache.clear();
    g_cache.emplace(key, code);
    return VEGAS_OK;
}

}  // namespace vegas
