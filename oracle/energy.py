"""Discrete grid energy and brute-force minimisation (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The energy of a labeling x of a 4-connected W x H grid is (Sec. 2.2,
eq. energy-pairwise, with the stereo discretisation f_ij = w_ij r(u_i - u_j)):

    E(x) = sum_i theta_i(x_i) + sum_{horizontal ij} w_h rho(x_i - x_j)
                              + sum_{vertical ij}   w_v rho(x_i - x_j),

rho(t) = min(|t|, T).  Arrays: theta (H, W, K), w_h (H, W-1), w_v (H-1, W),
labels (H, W) integer.
"""
from __future__ import annotations

import itertools

import numpy as np

from .chain import rho

__all__ = ["grid_energy", "brute_force_min", "all_labelings_energy"]


def grid_energy(theta, w_h, w_v, T: int, labels) -> float:
    theta = np.asarray(theta, np.float64)
    x = np.asarray(labels, np.int64)
    H, W, K = theta.shape
    e = np.take_along_axis(theta, x[:, :, None], axis=2).sum()
    if W > 1:
        e += (np.asarray(w_h, np.float64) * rho(x[:, 1:] - x[:, :-1], T)).sum()
    if H > 1:
        e += (np.asarray(w_v, np.float64) * rho(x[1:, :] - x[:-1, :], T)).sum()
    return float(e)


def all_labelings_energy(theta, w_h, w_v, T: int):
    """Energies of all K^(H W) labelings (tiny grids only); returns (labelings, energies)."""
    theta = np.asarray(theta, np.float64)
    H, W, K = theta.shape
    n = H * W
    if K ** n > 2_000_000:
        raise ValueError("grid too large for enumeration")
    labs = np.array(list(itertools.product(range(K), repeat=n)), dtype=np.int64).reshape(-1, H, W)
    flat_theta = theta.reshape(n, K)
    e = flat_theta[np.arange(n)[None, :], labs.reshape(-1, n)].sum(axis=1)
    if W > 1:
        e = e + (np.asarray(w_h, np.float64)[None] * rho(labs[:, :, 1:] - labs[:, :, :-1], T)).sum(axis=(1, 2))
    if H > 1:
        e = e + (np.asarray(w_v, np.float64)[None] * rho(labs[:, 1:, :] - labs[:, :-1, :], T)).sum(axis=(1, 2))
    return labs, e


def brute_force_min(theta, w_h, w_v, T: int):
    """Exact minimum energy and one minimiser by enumeration."""
    labs, e = all_labelings_energy(theta, w_h, w_v, T)
    i = int(np.argmin(e))
    return float(e[i]), labs[i]
