"""TRW-S on the two-family decomposition, as a CPU quality reference (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

App. A.1 derives TRW-S from the decomposition of Sec. 2.3 (F: rows with unaries
theta - lambda, G: columns with unaries lambda): it visits one node i at a time and
maximises the dual min F + min G over lambda_i alone, by making the two families'
min-marginals at i equal (eq. TRW-S-update):

    lambda_i += (m^F_i - m^G_i) / 2,

where m^F_i is the min-marginal at i of i's row chain and m^G_i that of its column chain
(the sign follows this decomposition: F carries -lambda).  The updates are sequential;
after an update the min-marginal at the next node of a chain needs only one message step
(eq. msg-pass): the message from the visited side is extended by the updated node, the
message from the unvisited side is still valid because those nodes have not changed since
it was computed.  One iteration is a forward pass over the nodes in raster order followed
by a backward pass in the reverse order (the unit of the comparison figures: one
forward-backward pass of TRW-S against one Dual_MM iteration, equal updates per pixel).

Messages are kept unnormalised (the min-marginals are the plain definitions); a constant
offset in m^F_i - m^G_i would only shift lambda_i by a constant, which moves the same
constant between F and G and leaves the bound unchanged.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import chain, dmm
from .energy import grid_energy

__all__ = ["TRWSResult", "trws", "trws_iteration"]


def _msg(v, w, T):
    return chain.message(v[None], np.array([w]), T)[0]


def trws_iteration(theta, lam, w_h, w_v, T):
    """One forward + backward pass of TRW-S; returns the new lambda (a copy)."""
    theta = np.asarray(theta, np.float64)
    w_h = np.asarray(w_h, np.float64)
    w_v = np.asarray(w_v, np.float64)
    lam = np.array(lam, np.float64, copy=True)
    H, W, K = theta.shape
    # messages into each node: from the left / right along its row (family F), from above /
    # below along its column (family G)
    Lm = np.zeros((H, W, K)); Rm = np.zeros((H, W, K))
    Um = np.zeros((H, W, K)); Dm = np.zeros((H, W, K))
    for y in range(H):
        for x in range(W - 2, -1, -1):
            Rm[y, x] = _msg(Rm[y, x + 1] + theta[y, x + 1] - lam[y, x + 1], w_h[y, x], T)
    for x in range(W):
        for y in range(H - 2, -1, -1):
            Dm[y, x] = _msg(Dm[y + 1, x] + lam[y + 1, x], w_v[y, x], T)

    def update(y, x):
        mF = theta[y, x] - lam[y, x] + Lm[y, x] + Rm[y, x]
        mG = lam[y, x] + Um[y, x] + Dm[y, x]
        lam[y, x] += 0.5 * (mF - mG)

    # forward pass (raster order): extend the messages to the right and downwards
    for y in range(H):
        for x in range(W):
            update(y, x)
            if x + 1 < W:
                Lm[y, x + 1] = _msg(Lm[y, x] + theta[y, x] - lam[y, x], w_h[y, x], T)
            if y + 1 < H:
                Um[y + 1, x] = _msg(Um[y, x] + lam[y, x], w_v[y, x], T)
    # backward pass (reverse raster order): extend the messages to the left and upwards
    for y in range(H - 1, -1, -1):
        for x in range(W - 1, -1, -1):
            update(y, x)
            if x - 1 >= 0:
                Rm[y, x - 1] = _msg(Rm[y, x] + theta[y, x] - lam[y, x], w_h[y, x - 1], T)
            if y - 1 >= 0:
                Dm[y - 1, x] = _msg(Dm[y, x] + lam[y, x], w_v[y - 1, x], T)
    return lam


@dataclasses.dataclass
class TRWSResult:
    lam: np.ndarray
    lb_trace: np.ndarray      # lower bound min F + min G after each iteration
    energy_trace: np.ndarray  # energy of the argmin labeling of F's min-marginals after each iteration


def trws(theta, w_h, w_v, T: int, n_iters: int, lam0=None) -> TRWSResult:
    """n_iters TRW-S iterations from lambda = 0 (or lam0).  The labeling reported after
    each iteration is the argmin of F's normalized row min-marginals (lowest label on ties),
    the rule used for Dual_MM, so the two are comparable."""
    theta = np.asarray(theta, np.float64)
    lam = np.zeros_like(theta) if lam0 is None else np.array(lam0, np.float64, copy=True)
    lbs, es = [], []
    for _ in range(n_iters):
        lam = trws_iteration(theta, lam, w_h, w_v, T)
        lbs.append(dmm.lower_bound(theta, lam, w_h, w_v, T))
        mm = chain.min_marginals(theta - lam, np.asarray(w_h, np.float64), T, normalized=True)
        es.append(grid_energy(theta, w_h, w_v, T, np.argmin(mm, axis=2)))
    return TRWSResult(lam=lam, lb_trace=np.array(lbs), energy_trace=np.array(es))
