"""Comparison helpers shared by the GPU parity tests (no GPU needed to import)."""
from __future__ import annotations

import numpy as np

# Min-marginal tolerance: |gpu - oracle| <= MM_RTOL * max(|oracle|, S), S = cost range.
MM_RTOL = 1e-5


def cost_scale(theta) -> float:
    th = np.asarray(theta, np.float64)
    return float(max(th.max() - th.min(), 1e-12))


def minmarg_errors(mm_gpu, mm_ref, theta):
    S = cost_scale(theta)
    err = np.abs(np.asarray(mm_gpu, np.float64) - mm_ref)
    scale = np.maximum(np.abs(mm_ref), S)
    return err, err / scale


def check_labels(lab_gpu, lab_ref, mm_ref, theta):
    """Labels equal, except at pixels where the GPU label is an exact-cost tie of the
    oracle's min-marginals within the min-marginal tolerance.  Returns (n_diff, n_bad)."""
    lab_gpu = np.asarray(lab_gpu, np.int64)
    diff = lab_gpu != lab_ref
    if not diff.any():
        return 0, 0
    S = cost_scale(theta)
    ys, xs = np.nonzero(diff)
    vals = mm_ref[ys, xs, lab_gpu[ys, xs]]
    tol = MM_RTOL * np.maximum(S, np.abs(mm_ref[ys, xs]).max(axis=1))
    bad = int((vals > tol).sum())
    return int(diff.sum()), bad


def summarize(name, **kv):
    parts = [f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kv.items()]
    print(f"[parity] {name}: " + " ".join(parts), flush=True)
