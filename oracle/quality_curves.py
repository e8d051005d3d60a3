"""Lower bound and energy per iteration: Dual_MM with each minorant beside TRW-S (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The analogue of the paper's comparison figures (Fig. alg-uniform and Fig. alg-iterative): a
small stereo crop (40 x 40, 16 labels, truncated-linear regulariser), lower bounds and the
energies of the labelings the methods produce, per iteration, where one iteration is one
Dual_MM iteration (a horizontal and a vertical half-step) or one forward-backward pass of
TRW-S (the same number of updates per pixel).  The crop is synthetic (the generator of the
stereo workloads: random texture, piecewise-planar disparity, noise), its cost the truncated
3 x 3 SAD and its weights the contrast weights of the image.

Usage: python -m oracle.quality_curves [--size 40] [--labels 16] [--iters 30]
"""
from __future__ import annotations

import argparse
import time

import numpy as np

from . import cost_volume, dmm, trws

METHODS = ("naive", "iterative", "hierarchical", "uniform", "trws")


def crop(W=40, H=40, K=16, seed=7):
    import synth
    pair = synth.stereo_pair(W, H, K, seed=seed, segments=3, slope=0.05)
    theta = cost_volume.sad_cost_volume(pair.left, pair.right, K)
    w_h, w_v = cost_volume.contrast_weights(pair.left, lambda_pw=0.1, sigma_c=0.1)
    return theta, w_h, w_v


def curves(W=40, H=40, K=16, n_iters=30, seed=7, T=3, methods=METHODS, gammas=(0.25, 0.25, 1.0)):
    """{method: (lower bound after each iteration, energy of its labeling after each iteration)}."""
    theta, w_h, w_v = crop(W, H, K, seed)
    out = {}
    for m in methods:
        if m == "trws":
            r = trws.trws(theta, w_h, w_v, T, n_iters)
            out[m] = (r.lb_trace, r.energy_trace)
            continue
        lam = np.zeros_like(theta)
        lbs, es = [], []
        for _ in range(n_iters):
            r = dmm.solve_discrete(theta, w_h, w_v, T, 1, minorant=m, gammas=gammas, lam0=lam)
            lam = r.lam
            lbs.append(r.lower_bound)
            es.append(r.energy)
        out[m] = (np.array(lbs), np.array(es))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=40)
    ap.add_argument("--labels", type=int, default=16)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--seed", type=int, default=7)
    a = ap.parse_args()
    t0 = time.time()
    res = curves(a.size, a.size, a.labels, a.iters, a.seed)
    best_e = min(e.min() for _, e in res.values())
    print(f"# {a.size}x{a.size}, K={a.labels}, T=3, seed {a.seed}; lowest energy found {best_e:.4f}; "
          f"{time.time() - t0:.0f} s")
    print("# iteration | " + " | ".join(f"{m} LB / E" for m in res))
    for i in range(a.iters):
        print(f"{i + 1:3d} | " + " | ".join(f"{res[m][0][i]:.4f} / {res[m][1][i]:.4f}" for m in res))


if __name__ == "__main__":
    main()
