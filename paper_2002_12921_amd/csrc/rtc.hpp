// Runtime compilation of caller-supplied integrands (host side).
#pragma once

#include <string>

#include "vegas.h"

namespace vegas {

// Largest block of the runtime-compiled event kernel (its launch bound).
constexpr int kUserThreads = 512;

// Compiles the user-integrand kernels (k_user_rtc.hpp after `source`) for
// dimension d, precision prec (FP64 or FP32) and gfx950 with the runtime
// compiler; no device is needed.  On VEGAS_OK `code` holds the code object;
// `log` always holds the compiler's messages.  Compiled code objects are kept
// per (d, precision, source) for the process.
vegas_status rtc_compile(const char* source, int d, int prec, std::string& code, std::string& log);

}  // namespace vegas
