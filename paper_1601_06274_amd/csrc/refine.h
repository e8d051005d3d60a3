// refine.h - shared declarations of the refinement kernels (forward and adjoint).
#pragma once

#include "common.h"

namespace dm {

// Primal-dual state in FP64, one value per pixel for each array (edge arrays indexed
// by the edge's left / upper pixel).  FP64 because the non-convex iteration amplifies
// rounding differences over hundreds of iterations; the arrays are a few MB and stay
// in the caches, so the wider type costs little.
typedef double rfloat;

struct RefineState {
    rfloat* u;
    rfloat* ph;
    rfloat* pv;
    rfloat* qh;
    rfloat* qv;
};

struct RefineScalars {
    rfloat tau, sigma, h, eps, delta, beta_minus;
};

struct RefineLayout {
    size_t u0, sL, sR, state0, state1, total, plane;
    size_t tape_u0, tape_mask, mask_plane;  // keep_tape: u0 per warp, branch masks per iteration
};

RefineLayout refine_layout(const dm_shape& s, const dm_refine_params* p);

// Batched refinement: per-instance state, and the work tables of the launches.
struct RefBatchInst {
    const void* theta;
    const int* labels;
    const float* w_h;
    const float* w_v;
    float* u_out;
    RefineState S[2];
    rfloat* u0;
    rfloat* sL;
    rfloat* sR;
    int W, H, K;
};
struct RefChunk {      // pixels [start, start + count) of one instance
    int inst;
    long long start;
    int count;
};
struct RefTile {       // one fused-iteration tile (kFTX x kFTY outputs) of one instance
    int inst, bx, by;
};
void refine_tile_extent(int W, int H, int& nbx, int& nby);
hipError_t launch_batched_refine(const RefBatchInst* insts, const RefChunk* chunks, int n_chunks, const RefTile* tiles,
                                 int n_tiles, dm_dtype dt, const dm_refine_params& p, hipStream_t st);
RefineState state_at(char* base, size_t plane);
int validate_refine(const dm_shape& s, const dm_refine_params* p);
RefineScalars refine_scalars(const dm_refine_params& p);

}  // namespace dm
