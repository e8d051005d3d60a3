// dmm_tile.hip - one compiled (lanes per chain, labels per lane) tile of the chain sweep.
// Built once per tile with -DDM_TILE_G=<lanes> -DDM_TILE_L=<labels per lane>.
#include "batched_kernels.h"
#include "dmm_adjoint.h"

#if !defined(DM_TILE_G) || !defined(DM_TILE_L)
#error "DM_TILE_G and DM_TILE_L must be defined"
#endif

namespace dm {
template hipError_t launch_tile<DM_TILE_G, DM_TILE_L>(const SweepArgs&, dm_dtype, hipStream_t);
template hipError_t launch_adjoint_tile<DM_TILE_G, DM_TILE_L>(const AdjArgs&, dm_dtype, hipStream_t);
template hipError_t launch_batched_tile<DM_TILE_G, DM_TILE_L>(const BatchLaunch&, bool, dm_dtype, int, hipStream_t);
}  // namespace dm
