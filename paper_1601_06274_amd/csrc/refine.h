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
};

RefineLayout refine_layout(const dm_shape& s);
RefineState state_at(char* base, size_t plane);
int validate_refine(const dm_shape& s, const dm_refine_params* p);
RefineScalars refine_scalars(const dm_refine_params& p);

}  // namespace dm
