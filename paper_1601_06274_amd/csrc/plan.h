// plan.h - what every batched plan owns: device allocations and its captured graph.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

namespace dm {

// A plan object behind the opaque handle of dm_plan_batched / dm_plan_batched_grad:
// dm_run_batched replays `exec`, dm_plan_destroy deletes the object.
struct PlanBase {
    std::vector<void*> allocs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t device_bytes = 0;
    virtual ~PlanBase() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* p : allocs) (void)hipFree(p);
    }
    template <typename T>
    T* alloc(size_t count) {
        void* p = nullptr;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        allocs.push_back(p);
        device_bytes += bytes;
        return static_cast<T*>(p);
    }
};

}  // namespace dm
