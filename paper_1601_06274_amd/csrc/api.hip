// api.hip - status strings, error reporting and shared validation of the C ABI.
#include <string.h>

#include <mutex>
#include <vector>

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
    const unsigned long long vol = (unsigned long long)s.W * (unsigned long long)s.H * (unsigned long long)s.K * 4ull;
    DM_REQUIRE(vol <= 0xFE000000ull, DM_ERR_SHAPE, "W*H*K*4 = %llu bytes exceeds the 32-bit volume offset range", vol);
    return DM_OK;
}

// ------------------------------------------------------------------ profiler
namespace {
struct ProfRecord {
    int kind;
    double bytes;
    hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
unsigned g_prof_mask = 0;
std::vector<ProfRecord> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
void recycle_all() {
    for (auto& r : g_prof) {
        if (r.start) g_event_pool.push_back(r.start);
        if (r.stop) g_event_pool.push_back(r.stop);
    }
    g_prof.clear();
}
}  // namespace

bool profiler_on() { return g_prof_on; }

int profiler_begin(int kind, double bytes, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || !(g_prof_mask & (1u << kind))) return -1;
    ProfRecord r{kind, bytes, take_event(), take_event()};
    if (!r.start || !r.stop) return -1;
    if (hipEventRecord(r.start, s) != hipSuccess) return -1;
    g_prof.push_back(r);
    return (int)g_prof.size() - 1;
}

void profiler_end(int id, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (id < 0 || id >= (int)g_prof.size()) return;
    (void)hipEventRecord(g_prof[id].stop, s);
}

}  // namespace dm

extern "C" int dm_profiler_enable(unsigned kind_mask) {
    std::lock_guard<std::mutex> lk(dm::g_prof_mu);
    const bool on = kind_mask != 0;
    if (on) {
        for (auto& r : dm::g_prof) {
            (void)hipEventSynchronize(r.stop);
        }
        dm::recycle_all();
    }
    dm::g_prof_on = on;
    if (on) dm::g_prof_mask = kind_mask;
    return DM_OK;
}

extern "C" int dm_profiler_query(int kind, long long* launches, double* total_ms, double* alg_bytes) {
    std::lock_guard<std::mutex> lk(dm::g_prof_mu);
    long long n = 0;
    double ms = 0.0, bytes = 0.0;
    for (auto& r : dm::g_prof) {
        if (r.kind != kind) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) {
            dm::set_error("profiler: event synchronize failed");
            return DM_ERR_HIP;
        }
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) {
            dm::set_error("profiler: elapsed time failed");
            return DM_ERR_HIP;
        }
        ++n;
        ms += t;
        bytes += r.bytes;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (alg_bytes) *alg_bytes = bytes;
    return DM_OK;
}

extern "C" const char* dm_status_string(int status) {
    switch (status) {
        case DM_OK: return "DM_OK";
        case DM_ERR_NULL: return "DM_ERR_NULL: required pointer is NULL";
        case DM_ERR_SHAPE: return "DM_ERR_SHAPE: W, H or K out of range";
        case DM_ERR_PARAM: return "DM_ERR_PARAM: parameter out of range";
        case DM_ERR_DTYPE: return "DM_ERR_DTYPE: unknown dtype";
        case DM_ERR_WORKSPACE: return "DM_ERR_WORKSPACE: workspace missing or too small";
        case DM_ERR_UNSUPPORTED: return "DM_ERR_UNSUPPORTED: not compiled into this library";
        case DM_ERR_HIP: return "DM_ERR_HIP: HIP runtime error";
        default: return "unknown dm_status";
    }
}

extern "C" const char* dm_last_error_message(void) { return dm::g_last_error; }

extern "C" const char* dm_version(void) { return "dmatch 0.1 gfx950 wave64"; }
