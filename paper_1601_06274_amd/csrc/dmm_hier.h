// dmm_hier.h - hierarchical-minorant half-step (App. A.3.3), launched by the Dual_MM driver.
#pragma once

#include "dmm_kernels.h"

namespace dm {

// One half-step of the family described by `a` (as for the chain sweeps: theta null for
// the vertical family, lam_in / lam the dual read and written, opt the per-chain optima)
// with the hierarchical minorant.  a.msg and msg_right are two message volumes of the
// volume's size.  A workgroup of one or four waves per chain; K <= 256.
hipError_t launch_hier_half_step(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st);

// Algorithmic HBM bytes of one such launch.
double hier_half_step_bytes(const SweepArgs& a, dm_dtype dt);

}  // namespace dm
