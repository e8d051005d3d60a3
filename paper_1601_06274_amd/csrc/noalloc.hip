// noalloc.hip - dm_solve_discrete_noalloc: Dual_MM without a caller workspace.
//
// For callers that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid it).  The solver's scratch memory (message volume,
// chain optima, partial sums, labels when none are requested) lives in one file-scope
// device array of kScratchBytes; this entry point allocates nothing and runs exactly the
// kernels of dm_solve_discrete on that array.
//
// The array is one per GPU (each device holds its own copy at its own address for the
// life of the process).  In host code its name is only a host-side stand-in, so the
// device address is looked up once per device with hipGetSymbolAddress and only that
// address is ever passed on.  Every call on one GPU shares the array: calls that overlap
// in time on the same GPU (different streams, or threads) race and must be serialised by
// the caller.  Nothing in the array has to start at zero: dm_solve_discrete writes every
// scratch value before it reads it, as it does with an uninitialised caller workspace.
#include <mutex>

#include "common.h"

namespace dm {
namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on the first call on each device,
// with that device current).
int scratch_for_current_device(void** out) {
    int dev = -1;
    DM_HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DM_REQUIRE(dev >= 0 && dev < kMaxDevices, DM_ERR_UNSUPPORTED, "device %d beyond the %d supported", dev,
               kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        DM_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        DM_REQUIRE(p != nullptr, DM_ERR_HIP, "scratch array has no device address on device %d", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DM_OK;
}

}  // namespace
}  // namespace dm

extern "C" size_t dm_solve_discrete_noalloc_limit(void) { return dm::kScratchBytes; }

extern "C" int dm_solve_discrete_noalloc(const void* cost, dm_dtype cost_dtype, const float* w_h, const float* w_v,
                                         dm_shape s, const dm_discrete_params* p, int32_t* labels_out,
                                         float* minmarg_out, float* dual_inout, double* bounds_out,
                                         double* lb_trace_out, void* hip_stream) {
    dm::clear_error();
    const size_t need = dm_solve_discrete_workspace(s, cost_dtype, p);
    if (need == 0) {
        // invalid arguments: let the solver report them (it validates before using the workspace)
        return dm_solve_discrete(cost, cost_dtype, w_h, w_v, s, p, labels_out, minmarg_out, dual_inout, bounds_out,
                                 lb_trace_out, nullptr, 0, hip_stream);
    }
    DM_REQUIRE(need <= dm::kScratchBytes, DM_ERR_WORKSPACE,
               "this problem needs %zu bytes of scratch; the no-allocation entry point holds %zu "
               "(use dm_solve_discrete with a caller workspace)",
               need, dm::kScratchBytes);
    void* ws = nullptr;
    int st = dm::scratch_for_current_device(&ws);
    if (st != DM_OK) return st;
    return dm_solve_discrete(cost, cost_dtype, w_h, w_v, s, p, labels_out, minmarg_out, dual_inout, bounds_out,
                             lb_trace_out, ws, dm::kScratchBytes, hip_stream);
}
