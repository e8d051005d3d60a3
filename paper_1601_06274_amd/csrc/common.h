// common.h - host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include "../../include/dmatch.h"

namespace dm {

// Thread-local detail for dm_last_error_message().
void set_error(const char* fmt, ...);
void clear_error();

// Converts a pending HIP error (sticky or from the last launch) into DM_ERR_HIP.
int check_hip(const char* where);

#define DM_REQUIRE(cond, code, ...)            \
    do {                                       \
        if (!(cond)) {                         \
            ::dm::set_error(__VA_ARGS__);      \
            return (code);                     \
        }                                      \
    } while (0)

#define DM_HIP_TRY(expr, where)                                                           \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::dm::set_error("%s: %s (%s)", (where), hipGetErrorName(e_), hipGetErrorString(e_)); \
            return DM_ERR_HIP;                                                            \
        }                                                                                 \
    } while (0)

int validate_shape(const dm_shape& s);

// Contrast edge weights w = lambda_pw * exp(-|I(neighbour) - I| / contrast_sigma) of one
// image (cost_volume.hip); w_h / w_v may be null.
hipError_t launch_contrast_weights(const float* I, int W, int H, float lambda_pw, float contrast_sigma, float* w_h,
                                   float* w_v, hipStream_t stream);
int validate_discrete(const dm_shape& s, const dm_discrete_params* p);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Kernel profiler (see dm_profiler_enable).  Usage around a launch:
//     ProfScope ps(DM_PROF_SWEEP_H, bytes, stream);  launch(...);  ps.stop();
bool profiler_on();
int profiler_begin(int kind, double bytes, hipStream_t s);   // returns record id or -1
void profiler_end(int id, hipStream_t s);

struct ProfScope {
    int id;
    hipStream_t s;
    ProfScope(int kind, double bytes, hipStream_t st) : id(profiler_on() ? profiler_begin(kind, bytes, st) : -1), s(st) {}
    void stop() {
        if (id >= 0) profiler_end(id, s);
        id = -1;
    }
    ~ProfScope() { stop(); }
};

}  // namespace dm
