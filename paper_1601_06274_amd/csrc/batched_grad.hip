// batched_grad.hip - many instances, each its own chain of kernels, as one captured graph.
//
// The differentiation workload: every instance runs Dual_MM keeping what its backward
// needs (Sec. 2.3, Alg. Dual_MM), the refinement keeping its prox branches (Sec. 2.4,
// Sec. 3.1), then the refinement adjoint and the Dual_MM adjoint; without gradient
// buffers, the forward only (Dual_MM and refinement).  One instance's chain families fill
// only part of the chip, so the instances run on forked streams of one graph: each
// instance's kernels form a chain of their own, and instances advance through their
// half-steps independently (no barrier common to all instances).  Instances go to the
// streams largest first, each to the stream with the least work so far (work ~ W*H*K);
// those of one stream run one after another and share that stream's workspaces.
#include <algorithm>
#include <string>
#include <vector>

#include "common.h"
#include "plan.h"

namespace dm {
namespace {

struct GradPlan : PlanBase {};

struct StreamWs {
    char *fwd = nullptr, *bwd = nullptr, *ref = nullptr, *refb = nullptr;
    size_t fwd_b = 0, bwd_b = 0, ref_b = 0, refb_b = 0;
};

}  // namespace
}  // namespace dm

using namespace dm;

extern "C" int dm_plan_batched_grad(const dm_grad_instance* inst, int n, dm_dtype cost_dtype,
                                    const dm_discrete_params* p, const dm_refine_params* rp, int n_streams,
                                    void** plan_out) {
    clear_error();
    DM_REQUIRE(plan_out != nullptr && inst != nullptr && p != nullptr, DM_ERR_NULL, "inst, params and plan_out required");
    *plan_out = nullptr;
    DM_REQUIRE(n >= 1 && n <= 4096, DM_ERR_PARAM, "n=%d instances out of range [1, 4096]", n);
    DM_REQUIRE(n_streams >= 1 && n_streams <= 16, DM_ERR_PARAM, "n_streams=%d out of range [1, 16]", n_streams);
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown cost dtype");
    DM_REQUIRE(p->warm_start == 0, DM_ERR_UNSUPPORTED, "batched gradient plans start every run from dual 0");
    // with gradients every instance has grad_cost; forward only: none has
    const bool grad = inst[0].grad_cost != nullptr;
    DM_REQUIRE(!grad || p->keep_checkpoints == 1 || p->keep_checkpoints == 2, DM_ERR_PARAM,
               "the forward must keep checkpoints for the backward (keep_checkpoints 1 or 2)");
    dm_refine_params rq{};
    if (rp != nullptr) {
        rq = *rp;
        rq.keep_tape = grad ? 1 : 0;  // the refinement adjoint reads the forward's branch tape
    }
    const int S = n_streams < n ? n_streams : n;
    // streams by work, largest instance first to the least loaded stream
    std::vector<int> order(n), stream_of(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto work = [&](int i) { return (double)inst[i].s.W * inst[i].s.H * inst[i].s.K; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    std::vector<double> load(S, 0.0);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        stream_of[i] = k;
        load[k] += work(i);
    }
    std::vector<StreamWs> ws(S);
    for (int i = 0; i < n; ++i) {
        const dm_grad_instance& I = inst[i];
        DM_REQUIRE(I.cost != nullptr && I.dual != nullptr && I.labels != nullptr, DM_ERR_NULL,
                   "instance %d: cost, dual and labels are required", i);
        DM_REQUIRE((I.grad_cost != nullptr) == grad, DM_ERR_NULL,
                   "instance %d: grad_cost must be given for every instance or for none", i);
        DM_REQUIRE(rp == nullptr || I.u != nullptr, DM_ERR_NULL, "instance %d: u required with refinement", i);
        const size_t f = dm_solve_discrete_workspace(I.s, cost_dtype, p);
        if (f == 0) {
            const std::string why = dm_last_error_message();
            set_error("instance %d: %s", i, why.c_str());
            return DM_ERR_PARAM;
        }
        StreamWs& w = ws[stream_of[i]];
        w.fwd_b = std::max(w.fwd_b, f);
        if (grad) w.bwd_b = std::max(w.bwd_b, dm_solve_discrete_backward_workspace(I.s, p));
        if (rp != nullptr) {
            w.ref_b = std::max(w.ref_b, dm_refine_continuous_workspace(I.s, &rq));
            if (grad) w.refb_b = std::max(w.refb_b, dm_refine_continuous_backward_workspace(I.s, &rq));
        }
    }
    hipError_t e0 = hipGetLastError();
    DM_REQUIRE(e0 == hipSuccess, DM_ERR_HIP, "pending HIP error before dm_plan_batched_grad: %s",
               hipGetErrorString(e0));

    auto plan = new (std::nothrow) GradPlan();
    DM_REQUIRE(plan != nullptr, DM_ERR_HIP, "out of host memory");
    auto fail_hip = [&](const char* what, hipError_t e) {
        set_error("dm_plan_batched_grad: %s: %s", what, hipGetErrorString(e));
        delete plan;
        return DM_ERR_HIP;
    };
    for (StreamWs& w : ws) {
        w.fwd = plan->alloc<char>(w.fwd_b);
        if (!w.fwd) return fail_hip("workspace allocation", hipErrorOutOfMemory);
        if (grad && !(w.bwd = plan->alloc<char>(w.bwd_b))) return fail_hip("workspace allocation", hipErrorOutOfMemory);
        if (rp != nullptr) {
            w.ref = plan->alloc<char>(w.ref_b);
            if (!w.ref) return fail_hip("workspace allocation", hipErrorOutOfMemory);
            if (grad && !(w.refb = plan->alloc<char>(w.refb_b)))
                return fail_hip("workspace allocation", hipErrorOutOfMemory);
        }
    }

    // capture: fork the instances over the side streams, join on the main stream
    hipStream_t main_s = nullptr;
    std::vector<hipStream_t> side(S, nullptr);
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join(S, nullptr);
    auto destroy = [&]() {
        if (main_s) (void)hipStreamDestroy(main_s);
        for (auto s2 : side)
            if (s2) (void)hipStreamDestroy(s2);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        for (auto ev : ev_join)
            if (ev) (void)hipEventDestroy(ev);
    };
    hipError_t e = hipStreamCreateWithFlags(&main_s, hipStreamNonBlocking);
    for (int k = 0; k < S && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
    for (int k = 0; k < S && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ev_join[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(main_s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        destroy();
        return fail_hip("streams / capture", e);
    }
    int st = DM_OK;
    hipError_t ce = hipEventRecord(ev_fork, main_s);
    for (int k = 0; k < S && ce == hipSuccess; ++k) ce = hipStreamWaitEvent(side[k], ev_fork, 0);
    for (int i = 0; i < n && st == DM_OK && ce == hipSuccess; ++i) {
        const dm_grad_instance& I = inst[i];
        const StreamWs& w = ws[stream_of[i]];
        void* s2 = side[stream_of[i]];
        st = dm_solve_discrete(I.cost, cost_dtype, I.w_h, I.w_v, I.s, p, I.labels, I.minmarg, I.dual, I.bounds,
                               nullptr, w.fwd, w.fwd_b, s2);
        if (st == DM_OK && rp != nullptr) {
            st = dm_refine_continuous(I.cost, cost_dtype, I.labels, I.w_h, I.w_v, I.s, &rq, I.u, w.ref, w.ref_b, s2);
            if (st == DM_OK && grad && I.grad_u != nullptr)
                st = dm_refine_continuous_backward(I.grad_u, I.cost, cost_dtype, I.w_h, I.w_v, I.s, &rq, w.ref, w.ref_b,
                                                   I.grad_cost, I.grad_w_h, I.grad_w_v, 0, w.refb, w.refb_b, s2);
        }
        const int acc = (rp != nullptr && I.grad_u != nullptr) ? 1 : 0;
        if (st == DM_OK && grad)
            st = dm_solve_discrete_backward(I.grad_minmarg, I.grad_bounds, I.cost, cost_dtype, I.w_h, I.w_v, I.s, p,
                                            I.dual, w.fwd, w.fwd_b, I.grad_cost, I.grad_w_h, I.grad_w_v, acc, w.bwd,
                                            w.bwd_b, s2);
    }
    for (int k = 0; k < S && ce == hipSuccess; ++k) {
        ce = hipEventRecord(ev_join[k], side[k]);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(main_s, ev_join[k], 0);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(main_s, &graph);
    destroy();
    if (st != DM_OK || ce != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st != DM_OK) {
            // keep the failing call's message
            delete plan;
            return st;
        }
        return fail_hip("capture", ce != hipSuccess ? ce : e);
    }
    plan->graph = graph;
    if ((e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0)) != hipSuccess)
        return fail_hip("instantiate", e);
    *plan_out = static_cast<PlanBase*>(plan);
    return DM_OK;
}
