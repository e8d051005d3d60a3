// dmm_tile.hip - one compiled (lanes per chain, labels per lane) tile of the chain sweeps.
// Built once per tile and part with -DDM_TILE_G=<lanes> -DDM_TILE_L=<labels per lane>
// and -DDM_TILE_PART=<1: forward sweeps, 2: adjoint sweeps (recomputing the selections),
// 3: batched sweeps, 4: adjoint sweeps reading the selection tape>, so the large
// instantiations compile in parallel.
#if !defined(DM_TILE_G) || !defined(DM_TILE_L) || !defined(DM_TILE_PART)
#error "DM_TILE_G, DM_TILE_L and DM_TILE_PART must be defined"
#endif

#if DM_TILE_PART == 1
#include "dmm_kernels.h"
namespace dm {
template hipError_t launch_tile<DM_TILE_G, DM_TILE_L>(const SweepArgs&, dm_dtype, hipStream_t);
}  // namespace dm
#elif DM_TILE_PART == 2
#include "dmm_adjoint.h"
namespace dm {
template hipError_t launch_adjoint_tile<DM_TILE_G, DM_TILE_L, false>(const AdjArgs&, dm_dtype, hipStream_t);
}  // namespace dm
#elif DM_TILE_PART == 4
#include "dmm_adjoint.h"
namespace dm {
template hipError_t launch_adjoint_tile<DM_TILE_G, DM_TILE_L, true>(const AdjArgs&, dm_dtype, hipStream_t);
}  // namespace dm
#elif DM_TILE_PART == 3
#include "batched_kernels.h"
namespace dm {
template hipError_t launch_batched_tile<DM_TILE_G, DM_TILE_L>(const BatchLaunch&, bool, dm_dtype, int, hipStream_t);
}  // namespace dm
#else
#error "unknown DM_TILE_PART"
#endif
