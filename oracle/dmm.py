"""Dual decomposition of the grid energy and the Dual_MM loop (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Decomposition (Sec. 2.3, eq. energy-chain-chain and DD-dual).  The grid
energy is split into a horizontal family F (all rows, pairwise weights w_h)
and a vertical family G (all columns, weights w_v).  A dual vector
lambda in R^{H x W x K} moves unary cost between them:

    F has unaries theta - lambda,  G has unaries lambda,

so F(x) + G(x) = E(x) for every labeling and every lambda, and
LB(lambda) = min F + min G <= min E (weak duality, Sec. 2.3).

Dual_MM (Sec. 2.3, Alg. Dual_MM) alternates two half-steps.  In the
horizontal half-step every row chain of F computes a modular minorant h of
itself and hands it to G (lambda += h); in the vertical half-step every
column chain of G computes its minorant and hands it to F (lambda -= h).
Chains within a half-step are independent.  With the minorant's exactness
(it keeps the chain optimum in the remainder, h >= 0) the lower bound does
not decrease (monotone block-coordinate ascent, Sec. 2.3).

Readings of the paper used here (the paper leaves them open):
  * start from lambda = 0 (all unary cost in F) unless a warm start is given,
    and take the horizontal half-step first;
  * one "dual iteration" is one horizontal plus one vertical half-step;
  * the output labeling is the argmin of the normalized row min-marginals of
    F after the last half-step (Alg. Dual_MM, minimisation step), ties going
    to the lowest label.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import chain
from .energy import grid_energy

__all__ = ["DMMResult", "lower_bound", "row_optima", "col_optima", "half_step", "solve_discrete"]


def _rows(vol):
    return vol  # (H, W, K): chains along axis 1


def _cols(vol):
    return np.ascontiguousarray(np.transpose(vol, (1, 0, 2)))  # (W, H, K)


def _minorant(a, w, T, minorant, gammas):
    if minorant == "iterative":
        return chain.iterative_minorant(a, w, T, gammas)
    if minorant == "naive":
        return chain.naive_minorant(a, w, T)
    if minorant == "hierarchical":
        return chain.hierarchical_minorant(a, w, T)
    if minorant == "uniform":
        return chain.uniform_minorant(a, w, T)
    raise ValueError(minorant)


def _chain_optima(a, w, T):
    """Optimum of every chain of a (C, n, K): min over labels of any min-marginal."""
    m = chain.min_marginals(a, w, T, normalized=False)
    return m[:, 0, :].min(axis=1)


def row_optima(theta, lam, w_h, T):
    """Optimum of each row chain of F (unaries theta - lambda)."""
    a = np.asarray(theta, np.float64) - lam
    return _chain_optima(a, np.asarray(w_h, np.float64), T)


def col_optima(lam, w_v, T):
    """Optimum of each column chain of G (unaries lambda)."""
    return _chain_optima(_cols(lam), np.asarray(w_v, np.float64).T, T)


def lower_bound(theta, lam, w_h, w_v, T) -> float:
    """Dual objective min F + min G (Sec. 2.3, eq. DD-dual)."""
    return float(row_optima(theta, lam, w_h, T).sum() + col_optima(lam, w_v, T).sum())


def half_step(theta, lam, w_h, w_v, T, family, minorant="iterative", gammas=(0.25, 0.25, 1.0)):
    """One half-step of Dual_MM on a copy of lambda; ``family`` is 'h' or 'v'."""
    theta = np.asarray(theta, np.float64)
    lam = np.array(lam, dtype=np.float64, copy=True)
    if family == "h":
        h = _minorant(theta - lam, np.asarray(w_h, np.float64), T, minorant, gammas)
        lam += h
    elif family == "v":
        h = _minorant(_cols(lam), np.asarray(w_v, np.float64).T, T, minorant, gammas)
        lam -= np.transpose(h, (1, 0, 2))
    else:
        raise ValueError(family)
    return lam


@dataclasses.dataclass
class DMMResult:
    labels: np.ndarray      # (H, W) int64
    minmarg: np.ndarray     # (H, W, K) normalized row min-marginals of F
    lam: np.ndarray         # (H, W, K) final dual point
    lower_bound: float      # min F + min G at the final lambda
    energy: float           # E(labels)
    lb_trace: np.ndarray    # LB after each half-step (length 2 n_iters, or n_half_steps)


def solve_discrete(theta, w_h, w_v, T: int, n_iters: int, *, minorant: str = "iterative",
                   gammas=(0.25, 0.25, 1.0), lam0=None, n_half_steps: int | None = None) -> DMMResult:
    """Run Dual_MM for ``n_iters`` dual iterations (or ``n_half_steps`` half-steps)."""
    theta = np.asarray(theta, np.float64)
    H, W, K = theta.shape
    lam = np.zeros_like(theta) if lam0 is None else np.array(lam0, dtype=np.float64, copy=True)
    steps = 2 * n_iters if n_half_steps is None else n_half_steps
    trace = []
    for s in range(steps):
        lam = half_step(theta, lam, w_h, w_v, T, "h" if s % 2 == 0 else "v", minorant, gammas)
        trace.append(lower_bound(theta, lam, w_h, w_v, T))
    mm = chain.min_marginals(theta - lam, np.asarray(w_h, np.float64), T, normalized=True)
    labels = np.argmin(mm, axis=2)           # numpy argmin returns the lowest index on ties
    return DMMResult(
        labels=labels,
        minmarg=mm,
        lam=lam,
        lower_bound=lower_bound(theta, lam, w_h, w_v, T),
        energy=grid_energy(theta, w_h, w_v, T, labels),
        lb_trace=np.array(trace),
    )
