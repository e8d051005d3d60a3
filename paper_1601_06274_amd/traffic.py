"""HBM traffic of a kernel from rocprofv3 counter runs.

Two `rocprofv3 --pmc` runs of the same program, one collecting FETCH_SIZE and one
WRITE_SIZE (KiB per dispatch, counted at the L2 / memory interface), give the bytes a
kernel moves.  Both counters are scaled by what they read for a plain elementwise
kernel of known size in the same run (`bench.py --traffic-probe` runs one: an in-place
multiply by 1 over a 1 GiB FP32 buffer, reading and writing 1 GiB), which absorbs the
counters' units and any fixed bias.

A launch of several dispatches of one kernel (the hierarchical half-step split into a
block per chain for the top levels and a block per subtree below) is counted with
`--per-launch n`: the mean over the dispatches times n.

Usage:
    python -m paper_1601_06274_amd.traffic --fetch F.csv --write W.csv --copy-bytes N \\
        --kernel <substring of the kernel name> [--per-launch n] [--out file.json]
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_KERNEL = "MulFunctor"


SOURCES = {"sweep": ["dmm_kernels.h", "wave.h", "tiles.h"],
           "adjoint": ["dmm_kernels.h", "wave.h", "tiles.h", "dmm_adjoint.h"],
           "hier": ["dmm_hier.hip", "dmm_hier.h"]}


def source_hash(which: str = "sweep") -> str:
    """Hash of the sources of the chain sweep ("sweep"), adjoint ("adjoint") or
    hierarchical-minorant ("hier") kernels (a stored traffic figure is valid only for the
    kernel it was measured on)."""
    h = hashlib.sha256()
    for fn in SOURCES[which]:
        with open(os.path.join(HERE, "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _per_dispatch(path: str, counter: str) -> dict[str, list[float]]:
    """Kernel name -> counter value of each dispatch."""
    out: dict[str, list[float]] = {}
    with open(path, newline="") as f:
        rows = list(csv.DictReader(f))
    if not rows:
        raise ValueError(f"{path}: no rows")
    keys = rows[0].keys()
    kname = next(k for k in keys if k.lower() in ("kernel_name", "kernel-name", "name"))
    cname = next(k for k in keys if k.lower() in ("counter_name", "counter-name"))
    cval = next(k for k in keys if k.lower() in ("counter_value", "counter-value", "value"))
    for r in rows:
        if r[cname] != counter:
            continue
        out.setdefault(r[kname], []).append(float(r[cval]))
    return out


def _median_for(d: dict[str, list[float]], sub: str) -> tuple[float, int, str]:
    names = [k for k in d if sub in k]
    if not names:
        raise KeyError(f"no kernel matching {sub!r}")
    vals = [v for k in names for v in d[k]]
    return statistics.median(vals), len(vals), names[0]


def _per_launch_for(d: dict[str, list[float]], sub: str, n: int) -> tuple[float, int, str]:
    """Mean over the matching dispatches times n (a launch of n dispatches)."""
    names = [k for k in d if sub in k]
    if not names:
        raise KeyError(f"no kernel matching {sub!r}")
    vals = [v for k in names for v in d[k]]
    if len(vals) % n:
        raise ValueError(f"{len(vals)} dispatches of {sub!r} are not whole launches of {n}")
    return statistics.fmean(vals) * n, len(vals), names


def summarize(fetch_csv: str, write_csv: str, copy_bytes: float, kernel: str, sources: str = "sweep",
              per_launch: int = 1) -> dict:
    fd = _per_dispatch(fetch_csv, "FETCH_SIZE")
    wd = _per_dispatch(write_csv, "WRITE_SIZE")
    pf, _, _ = _median_for(fd, PROBE_KERNEL)
    pw, _, _ = _median_for(wd, PROBE_KERNEL)
    if per_launch > 1:
        kf, nf, names = _per_launch_for(fd, kernel, per_launch)
        kw, nw, _ = _per_launch_for(wd, kernel, per_launch)
        name = names[0]
    else:
        kf, nf, name = _median_for(fd, kernel)
        kw, nw, _ = _median_for(wd, kernel)
        names = [name]
    sf = copy_bytes / pf  # bytes per counter unit, from the probe
    sw = copy_bytes / pw
    return {
        "kernel": name,
        "kernels_matched": names,
        "sources": sources,
        "kernel_source_hash": source_hash(sources),
        "dispatches": [nf, nw],
        "dispatches_per_launch": per_launch,
        "fetch_kib_raw": kf,
        "write_kib_raw": kw,
        "probe_fetch_kib_raw": pf,
        "probe_write_kib_raw": pw,
        "probe_bytes": copy_bytes,
        "scale_fetch": sf / 1024.0,
        "scale_write": sw / 1024.0,
        "fetch_bytes_per_launch": kf * sf,
        "write_bytes_per_launch": kw * sw,
        "bytes_per_launch": kf * sf + kw * sw,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--sources", default="sweep", choices=sorted(SOURCES))
    ap.add_argument("--per-launch", type=int, default=1)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = summarize(a.fetch, a.write, a.copy_bytes, a.kernel, a.sources, a.per_launch)
    txt = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt)
    return 0


if __name__ == "__main__":
    sys.exit(main())
