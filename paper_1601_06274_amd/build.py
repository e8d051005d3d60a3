"""Builds libdmatch.so for gfx950 in place (hipcc, no torch extension machinery).

Usage: python -m paper_1601_06274_amd.build [--jobs N] [--incremental]

By default every unit is compiled.  With --incremental a unit is skipped when its object
is newer than every file its last compile depended on (hipcc's dependency list, kept
beside the object).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdmatch.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, extra defines, object name)
def _tiles():
    """The tile list of csrc/tiles.h (one compilation unit per tile)."""
    with open(os.path.join(CSRC, "tiles.h")) as f:
        return [(int(g), int(l)) for g, l in re.findall(r"X\((\d+),\s*(\d+)\)", f.read())]


TILES = _tiles()
UNITS = [("api.hip", [], "api"), ("dmm.hip", [], "dmm"), ("cost_volume.hip", [], "cost_volume"),
         ("refine.hip", [], "refine"), ("batched.hip", [], "batched"), ("noalloc.hip", [], "noalloc"), ("batched_grad.hip", [], "batched_grad"),
         ("flow.hip", [], "flow")]
# largest units first so the parallel build's critical path starts early
UNITS = [("dmm_tile.hip", [f"-DDM_TILE_G={g}", f"-DDM_TILE_L={l}", f"-DDM_TILE_PART={k}"], f"dmm_tile_{g}x{l}_{v}")
         for k, v in [(2, "adj"), (4, "tape"), (1, "fwd"), (3, "batch")] for g, l in sorted(TILES, key=lambda t: -t[0] * t[1])] + UNITS
# the hierarchical-minorant kernels, one unit per labels-per-lane count (the slowest
# compiles: first), and their dispatch
UNITS = ([("dmm_hier.hip", [f"-DDM_HIER_LPL={l}"], f"dmm_hier_{l}") for l in (3, 4, 2, 1)] + UNITS +
         [("dmm_hier.hip", ["-DDM_HIER_LPL=0"], "dmm_hier_0")])

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fno-honor-nans",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wno-unused-result",
    # device code objects stored compressed (zstd) in the library, unpacked by the HIP
    # runtime at load: about a third of the size
    "--offload-compress",
]


def _up_to_date(obj: str, dep: str) -> bool:
    """True when `obj` is newer than every prerequisite listed in the make-style `dep`."""
    if not (os.path.exists(obj) and os.path.exists(dep)):
        return False
    with open(dep) as f:
        text = f.read().replace("\\\n", " ")
    _, _, prereqs = text.partition(":")
    t = os.path.getmtime(obj)
    for p in prereqs.split():
        if not os.path.exists(p) or os.path.getmtime(p) > t:
            return False
    return True


def _compile(unit, incremental=False) -> str:
    src, defs, name = unit
    obj = os.path.join(BUILD, name + ".o")
    dep = os.path.join(BUILD, name + ".d")
    if incremental and _up_to_date(obj, dep):
        return obj
    cmd = [HIPCC, *FLAGS, *defs, "-MMD", "-MF", dep, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1)
    for f in os.listdir(BUILD):  # objects of units that no longer exist
        if f.endswith(".o") and f[:-2] not in {u[2] for u in UNITS}:
            os.remove(os.path.join(BUILD, f))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, incremental), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true", help="skip units whose object is up to date")
    a = ap.parse_args()
    build(a.jobs, verbose=True, incremental=a.incremental)
    sys.exit(0)
