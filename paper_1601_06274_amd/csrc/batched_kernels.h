// batched_kernels.h - persistent work-queue form of the chain sweep for many instances.
//
// One launch processes one half-step (or the final row pass) of every instance whose
// labels count maps to this tile.  A fixed grid of single-wave workers pulls work items
// (instance, first chain of a lane group) from an atomic counter; items are ordered by
// decreasing chain length so the longest chains start first (uneven instances balance).
// There is no dependency between items of one launch, so the queue needs no waiting;
// half-step ordering is given by the launch sequence, which the plan captures once into
// a hipGraph.
#pragma once

#include "dmm_kernels.h"

namespace dm {

struct InstDesc {
    const void* theta;      // [H][W][K] cost
    float* lam;             // [H][W][K] dual
    float* msg;             // [H][W][K] message scratch
    const float* w_h;       // [H][W-1]
    const float* w_v;       // [H-1][W]
    int* labels;            // [H][W]
    double* opt_rows;       // [H] row chain optima (plan scratch; null without bounds)
    double* opt_cols;       // [W] column chain optima
    double* bounds;         // [2] = {LB, E(labels)} or null
    float* minmarg;         // [H][W][K] final-pass min-marginals or null
    int W, H, K;
    unsigned vol_bytes_f32, vol_bytes_theta, wh_bytes, wv_bytes;
};

struct BatchItem {
    int inst;   // instance index
    int chain;  // first chain of the lane group
};

struct BatchLaunch {
    const InstDesc* insts;
    const BatchItem* items;
    int n_items;
    int* counter;           // zeroed before the launch
    int family;             // 0: rows (horizontal), 1: columns (vertical)
    int mode, T, n_pass;
    int want_opt;           // store each chain's optimum into opt_rows / opt_cols
    float gamma[8];
};

__device__ __forceinline__ SweepArgs batch_args(const InstDesc& in, const BatchLaunch& bl) {
    SweepArgs a{};
    const bool rows = bl.family == 0;
    a.theta = rows ? in.theta : nullptr;
    a.lam = in.lam;
    a.lam_in = in.lam;
    a.msg = in.msg;
    a.w = rows ? in.w_h : in.w_v;
    a.minmarg = bl.mode == kModeFinal ? in.minmarg : nullptr;
    a.labels = in.labels;
    a.opt = bl.want_opt ? (rows ? in.opt_rows : in.opt_cols) : nullptr;
    a.chain_px = rows ? in.W : 1;
    a.node_px = rows ? 1 : in.W;
    a.w_chain = rows ? in.W - 1 : 1;
    a.w_node = rows ? 1 : in.W;
    a.vol_bytes_f32 = in.vol_bytes_f32;
    a.vol_bytes_theta = in.vol_bytes_theta;
    a.w_bytes = rows ? in.wh_bytes : in.wv_bytes;
    a.K = in.K;
    a.n = rows ? in.W : in.H;
    a.n_chains = rows ? in.H : in.W;
    a.T = bl.T;
    a.mode = bl.mode;
    a.n_pass = bl.n_pass;
    a.sign = rows ? 1.0f : -1.0f;
    a.inv_n = 1.0f / (float)a.n;
#pragma unroll
    for (int i = 0; i < 8; ++i) a.gamma[i] = bl.gamma[i];
    return a;
}

template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA, int MG>
__global__ __launch_bounds__(64) void batched_sweep_kernel(BatchLaunch bl) {
    __shared__ int s_item;
    constexpr int CPW = 64 / G;
    const int lane = threadIdx.x;
    for (;;) {
        if (lane == 0) s_item = atomicAdd(bl.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= bl.n_items) break;  // every worker leaves once the queue is drained
        const BatchItem bi = bl.items[it];
        const InstDesc in = bl.insts[bi.inst];
        const SweepArgs a = batch_args(in, bl);
        run_chain<G, LPL, PF, TT, FULL, HAS_THETA, MG>(a, bi.chain + lane / G, lane % G);
        (void)CPW;
    }
}

template <int G, int LPL>
hipError_t launch_batched_tile(const BatchLaunch& bl, bool full, dm_dtype dt, int workers, hipStream_t st) {
    // family 0 reads the cost; the final pass is a row pass, the optimum pass a column pass
    const bool final_pass = bl.mode == kModeFinal;
    const bool opt_pass = bl.mode == kModeOptimum;
#define DM_BATCH_LAUNCH(TT, FULLV, HT, MGV)                                                                      \
    hipLaunchKernelGGL((batched_sweep_kernel<G, LPL, kPF, TT, FULLV, HT, MGV>), dim3(workers), dim3(64), 0, st, bl)
    if (bl.family == 0) {
        if (dt == DM_F16) {
            if (full) {
                if (final_pass) DM_BATCH_LAUNCH(_Float16, true, true, kGroupFinal);
                else DM_BATCH_LAUNCH(_Float16, true, true, kGroupHalfStep);
            } else {
                if (final_pass) DM_BATCH_LAUNCH(_Float16, false, true, kGroupFinal);
                else DM_BATCH_LAUNCH(_Float16, false, true, kGroupHalfStep);
            }
        } else {
            if (full) {
                if (final_pass) DM_BATCH_LAUNCH(float, true, true, kGroupFinal);
                else DM_BATCH_LAUNCH(float, true, true, kGroupHalfStep);
            } else {
                if (final_pass) DM_BATCH_LAUNCH(float, false, true, kGroupFinal);
                else DM_BATCH_LAUNCH(float, false, true, kGroupHalfStep);
            }
        }
    } else {
        if (full) {
            if (opt_pass) DM_BATCH_LAUNCH(float, true, false, kGroupOptimum);
            else DM_BATCH_LAUNCH(float, true, false, kGroupHalfStep);
        } else {
            if (opt_pass) DM_BATCH_LAUNCH(float, false, false, kGroupOptimum);
            else DM_BATCH_LAUNCH(float, false, false, kGroupHalfStep);
        }
    }
#undef DM_BATCH_LAUNCH
    return hipGetLastError();
}

}  // namespace dm
