"""MI355X (gfx950) library for discrete-continuous dense matching.

Hot path of Shekhovtsov, Reinbacher, Graber and Pock, "Solving Dense Image
Matching in Real-Time using Discrete-Continuous Optimization" (CVWW 2016):
a W x H x K cost volume, the Dual_MM discrete solver over horizontal and
vertical chains, and the continuous primal-dual refinement, all as hand-written
HIP kernels behind the C ABI of ``include/dmatch.h``.

The Python layer only marshals arguments (torch tensors for device memory and
streams).  Importing the package does not load the shared library; the first
call does, and it raises if ``libdmatch.so`` has not been built.
"""
from ._lib import DmError, lib  # noqa: F401
from .ops import (DiscreteResult, FlowResult, build_cost_volume, build_cost_volume_census,  # noqa: F401
                  build_flow_cost_volume, flow_project, lr_check, refine_continuous, refine_continuous_backward,
                  refine_flow, solve_discrete, solve_discrete_backward, solve_flow, tile_for)

__all__ = ["DmError", "lib", "DiscreteResult", "solve_discrete", "solve_discrete_backward", "tile_for",
           "refine_continuous", "refine_continuous_backward", "build_cost_volume", "build_cost_volume_census",
           "lr_check", "build_flow_cost_volume", "flow_project", "refine_flow", "solve_flow", "FlowResult"]
