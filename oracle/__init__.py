"""FP64 CPU oracle for the discrete-continuous matching hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU
baseline leg of ``bench.py`` use it.  It shares no code with the HIP library
(``paper_1601_06274_amd``) and imports nothing from it.

Everything here is a plain, slow, directly readable restatement of the paper
(Shekhovtsov, Reinbacher, Graber, Pock: "Solving Dense Image Matching in
Real-Time using Discrete-Continuous Optimization", CVWW 2016), computed in
float64 with numpy.  The only vectorisation is across chains that the paper
itself declares independent (all rows of one half-step, all columns of the
other); along a chain every step is taken in the paper's order.

Modules
  chain        messages, min-marginals, iterative / naive / hierarchical / uniform minorants (App. A.1, A.3)
  dmm          dual decomposition and the Dual_MM loop (Sec. 2.3, Alg. Dual_MM)
  energy       the discrete energy and brute-force minimisation (Sec. 2.2)
  cost_volume  SAD cost volume and contrast edge weights (Sec. 2.2 "Stereo", Sec. 3.1)
  census       Census + Hamming cost volume and the left-right check (Sec. 3.1)
  refine       continuous refinement by non-linear primal-dual (Sec. 2.4, Sec. 3.1)
  trws         TRW-S on the same decomposition (App. A.1, eq. TRW-S-update), a quality reference
  flow         optical flow: 2-D SAD cost, decoupled layer costs, quadratic-fit refinement (Sec. 2.2, 3.2)
"""
from . import chain, dmm, energy, cost_volume, census, refine, trws, flow  # noqa: F401
