// C-ABI runtime pieces: version, per-thread error text.
#include <cstdio>
#include <string>

#include "common.hpp"

namespace bfx {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string &msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char *what) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e),
                  (int)e);
    set_error(buf);
    return BFX_E_HIP;
}

}  // namespace bfx

extern "C" int bfx_version(void) { return 10000; }

extern "C" const char *bfx_last_error_string(void) {
    return bfx::g_last_error.c_str();
}
