"""Builds libdmatch.so for gfx950 in place (hipcc, no torch extension machinery).

Usage: python -m paper_1601_06274_amd.build [--jobs N]
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
         ("refine.hip", [], "refine"), ("batched.hip", [], "batched")]
# largest units first so the parallel build's critical path starts early
UNITS = [("dmm_tile.hip", [f"-DDM_TILE_G={g}", f"-DDM_TILE_L={l}", f"-DDM_TILE_PART={k}"], f"dmm_tile_{g}x{l}_{v}")
         for k, v in [(2, "adj"), (4, "tape"), (1, "fwd"), (3, "batch")] for g, l in sorted(TILES, key=lambda t: -t[0] * t[1])] + UNITS
# the hierarchical-minorant unit is the slowest single compile: first
UNITS = [("dmm_hier.hip", [], "dmm_hier")] + UNITS

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fno-honor-nans",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wno-unused-result",
]


def _compile(unit) -> str:
    src, defs, name = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1)
    for f in os.listdir(BUILD):  # objects of units that no longer exist
        if f.endswith(".o") and f[:-2] not in {u[2] for u in UNITS}:
            os.remove(os.path.join(BUILD, f))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, UNITS))
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
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
