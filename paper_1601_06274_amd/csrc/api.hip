// api.hip - status strings, error reporting and shared validation of the C ABI.
#include <string.h>

#include "common.h"

namespace dm {

static thread_local char g_last_error[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = '\0'; }

int check_hip(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s (%s)", where, hipGetErrorName(e), hipGetErrorString(e));
        return DM_ERR_HIP;
    }
    return DM_OK;
}

int validate_shape(const dm_shape& s) {
    DM_REQUIRE(s.W >= 1 && s.W <= 16384, DM_ERR_SHAPE, "W=%d out of range [1, 16384]", s.W);
    DM_REQUIRE(s.H >= 1 && s.H <= 16384, DM_ERR_SHAPE, "H=%d out of range [1, 16384]", s.H);
    DM_REQUIRE(s.K >= 1 && s.K <= 256, DM_ERR_SHAPE, "K=%d out of range [1, 256]", s.K);
    return DM_OK;
}

}  // namespace dm

extern "C" const char* dm_status_string(int status) {
    switch (status) {
        case DM_OK: return "DM_OK";
        case DM_ERR_NULL: return "DM_ERR_NULL: required pointer is NULL";
        case DM_ERR_SHAPE: return "DM_ERR_SHAPE: W, H or K out of range";
        case DM_ERR_PARAM: return "DM_ERR_PARAM: parameter out of range";
        case DM_ERR_DTYPE: return "DM_ERR_DTYPE: unknown dtype";
        case DM_ERR_WORKSPACE: return "DM_ERR_WORKSPACE: workspace missing or too small";
        case DM_ERR_UNSUPPORTED: return "DM_ERR_UNSUPPORTED: not supported by this build";
        case DM_ERR_HIP: return "DM_ERR_HIP: HIP runtime error";
        default: return "unknown dm_status";
    }
}

extern "C" const char* dm_last_error_message(void) { return dm::g_last_error; }

extern "C" const char* dm_version(void) { return "dmatch 0.1 gfx950 wave64"; }
