"""Optical flow: decoupled two-layer discrete stage and 2-D quadratic-fit refinement (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Flow (Sec. 2.2 "Flow", Sec. 3.2): u_i in R^2, labels are pairs of displacements.  The
discretised data cost of pixel i is a K1 x K2 table D_i(x1, x2) (label x1 <-> horizontal
displacement x1 - off1, x2 <-> vertical displacement x2 - off2).  The discrete stage
decouples the two components by optimistic unaries (eq. flow decoupled costs)

    f1_i(x1) = min_{x2} D_i(x1, x2),      f2_i(x2) = min_{x1} D_i(x1, x2),

and regularises each layer on its own, i.e. two independent stereo-like Dual_MM solves
on the same grid and edge weights.  The regulariser of the continuous problem is
separable over the components (eq. regularizer-form: sum over k of r((A u^k)_ij)), so
the refinement runs the primal-dual iteration of Sec. 2.4 on each component with its
own duals p^k, q^k; only the data term differs from stereo.  Around the current point
u0 it is the quadratic model (eq. quadfit)

    D~_i(u) = D_i(u0) + L_i^T (u - u0) + 1/2 (u - u0)^T Q_i (u - u0)  on the box u0 +- h,

with L_i and Q_i finite-difference approximations (step h) of the gradient and Hessian,
keeping only the positive-semidefinite part of Q_i.

Readings (the paper leaves these open or prints them garbled):
  * D_i between labels is the bilinear interpolation of the table, each argument clamped
    to its label range (the stereo path's linear interpolation, in two dimensions).
  * Q_i is taken diagonal - the two central second differences, each clamped at 0 (its
    positive-semidefinite part) - so that the prox is point-wise per component, as the
    paper writes it; L_i are the central first differences.  Arguments beyond the label
    range are clamped by the interpolation.
  * The prox of tau D~ (eq. prox_flow) is the minimiser of
    1/2 (v - u_hat)^2 + tau (L (v - u0) + Q/2 (v - u0)^2) over the box, per component:
        v = clamp(u0 +- h, (u_hat + tau (Q u0 - L)) / (1 + tau Q))
    The printed denominator 1 + tau L is read as 1 + tau Q (the stationarity condition
    of that quadratic); the box is also intersected with the label range, as for stereo.
  * A flow cost volume from images: the stereo SAD with a two-dimensional displacement,
    e(x, y, i, j) = |I1(x, y) - I2(x + i - off1, y + j - off2)| (tau outside I2),
    D[y][x][j][i] = min(tau, mean of e over the 3 x 3 window clamped to the image).
    (The paper's flow experiments reuse its stereo data term.)
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import dmm
from .refine import RefineParams, grad_op, grad_op_T, prox_conj

__all__ = ["flow_cost_volume", "project", "interp2", "linearize_quadfit", "prox_flow", "refine_flow",
           "solve_flow", "FlowResult"]


def flow_cost_volume(I1, I2, K1: int, K2: int, off1: int, off2: int, window: int = 3, trunc: float = 0.3,
                     rows=None):
    """[H][W][K2][K1] truncated windowed SAD between I1 at (x, y) and I2 at the displaced
    position (x + i - off1, y + j - off2); a displaced position outside I2 costs trunc.
    ``rows`` = (lo, hi) returns only the output rows lo..hi-1 (the same values)."""
    A = np.asarray(I1, np.float64)
    B = np.asarray(I2, np.float64)
    H, W = A.shape
    r = window // 2
    lo, hi = (0, H) if rows is None else rows
    ys_out = np.arange(lo, hi)
    e_rows = np.arange(max(lo - r, 0), min(hi + r, H))  # the rows of e the windows reach
    xs = np.arange(W)
    out = np.zeros((hi - lo, W, K2, K1))
    for j in range(K2):
        for i in range(K1):
            d1, d2 = i - off1, j - off2
            e = np.full((len(e_rows), W), trunc)
            vx = (xs + d1 >= 0) & (xs + d1 < W)
            vy = (e_rows + d2 >= 0) & (e_rows + d2 < H)
            yy, xx = np.nonzero(vy[:, None] & vx[None, :])
            e[yy, xx] = np.abs(A[e_rows[yy], xx] - B[e_rows[yy] + d2, xx + d1])
            acc = np.zeros((hi - lo, W))
            for dy in range(-r, r + 1):
                cy = np.clip(ys_out + dy, 0, H - 1) - e_rows[0]
                for dx in range(-r, r + 1):
                    cx = np.clip(xs + dx, 0, W - 1)
                    acc += e[cy][:, cx]
            out[:, :, j, i] = np.minimum(trunc, acc / float(window * window))
    return out


def project(D):
    """Optimistic decoupled unaries (eq. flow decoupled costs): f1 = min over x2, f2 = min over x1."""
    D = np.asarray(D, np.float64)
    return D.min(axis=2), D.min(axis=3)


def interp2(D, v1, v2):
    """D_i at continuous (v1, v2): bilinear interpolation of the table, arguments clamped."""
    D = np.asarray(D, np.float64)
    H, W, K2, K1 = D.shape
    v1 = np.clip(np.asarray(v1, np.float64), 0.0, K1 - 1.0)
    v2 = np.clip(np.asarray(v2, np.float64), 0.0, K2 - 1.0)
    a0 = np.minimum(np.floor(v1).astype(np.int64), K1 - 1)
    b0 = np.minimum(np.floor(v2).astype(np.int64), K2 - 1)
    a1 = np.minimum(a0 + 1, K1 - 1)
    b1 = np.minimum(b0 + 1, K2 - 1)
    t, s = v1 - a0, v2 - b0
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    d00, d01 = D[yy, xx, b0, a0], D[yy, xx, b0, a1]
    d10, d11 = D[yy, xx, b1, a0], D[yy, xx, b1, a1]
    return (1 - s) * ((1 - t) * d00 + t * d01) + s * ((1 - t) * d10 + t * d11)


def linearize_quadfit(D, u1, u2, h):
    """Gradient L and the positive part of the diagonal Hessian Q of the data term at
    (u1, u2), by central differences with step h (eq. quadfit)."""
    c = interp2(D, u1, u2)
    p1, m1 = interp2(D, u1 + h, u2), interp2(D, u1 - h, u2)
    p2, m2 = interp2(D, u1, u2 + h), interp2(D, u1, u2 - h)
    L1 = (p1 - m1) / (2.0 * h)
    L2 = (p2 - m2) / (2.0 * h)
    Q1 = np.maximum((p1 - 2.0 * c + m1) / (h * h), 0.0)
    Q2 = np.maximum((p2 - 2.0 * c + m2) / (h * h), 0.0)
    return L1, L2, Q1, Q2


def prox_flow(u_hat, u0, L, Q, tau, h, K):
    """prox of tau * D~ for one component (eq. prox_flow with the denominator 1 + tau Q)."""
    v = (u_hat + tau * (Q * u0 - L)) / (1.0 + tau * Q)
    lo = np.maximum(u0 - h, 0.0)
    hi = np.minimum(u0 + h, K - 1.0)
    return np.clip(v, lo, hi)


def refine_flow(D, w_h, w_v, labels1, labels2, params: RefineParams, *, return_state: bool = False):
    """Warped non-linear primal-dual refinement of both flow components (label units)."""
    D = np.asarray(D, np.float64)
    H, W, K2, K1 = D.shape
    w_h = np.asarray(w_h, np.float64)
    w_v = np.asarray(w_v, np.float64)
    P = params
    beta_minus = P.C + P.delta - P.eps * P.delta
    u = [np.asarray(labels1, np.float64).copy(), np.asarray(labels2, np.float64).copy()]
    st = [dict(ph=np.zeros((H, W - 1)), pv=np.zeros((H - 1, W)), qh=np.zeros((H, W - 1)), qv=np.zeros((H - 1, W)))
          for _ in range(2)]
    Kk = (K1, K2)
    for _ in range(P.n_warps):
        u0 = [u[0].copy(), u[1].copy()]
        L1, L2, Q1, Q2 = linearize_quadfit(D, u0[0], u0[1], P.h)
        LQ = ((L1, Q1), (L2, Q2))
        for _ in range(P.n_iters):
            for k in range(2):
                s = st[k]
                Lk, Qk = LQ[k]
                u_hat = u[k] - P.tau * grad_op_T(s["ph"] - s["qh"], s["pv"] - s["qv"], (H, W))
                u_new = prox_flow(u_hat, u0[k], Lk, Qk, P.tau, P.h, Kk[k])
                gh, gv = grad_op(u[k])
                s["qh"] = prox_conj(s["qh"] + P.tau * gh, w_h, 0.0, beta_minus, P.tau)
                s["qv"] = prox_conj(s["qv"] + P.tau * gv, w_v, 0.0, beta_minus, P.tau)
                bh, bv = grad_op(2.0 * u_new - u[k])
                s["ph"] = prox_conj(s["ph"] + P.sigma * bh, w_h, P.eps, P.delta, P.sigma)
                s["pv"] = prox_conj(s["pv"] + P.sigma * bv, w_v, P.eps, P.delta, P.sigma)
                u[k] = u_new
    if return_state:
        return u[0], u[1], st
    return u[0], u[1]


@dataclasses.dataclass
class FlowResult:
    f1: np.ndarray
    f2: np.ndarray
    layer1: dmm.DMMResult
    layer2: dmm.DMMResult
    u1: np.ndarray
    u2: np.ndarray


def solve_flow(D, w_h, w_v, T: int, n_iters: int, params: RefineParams, **dmm_kw) -> FlowResult:
    """Decoupled costs, one Dual_MM solve per layer, then the quadratic-fit refinement."""
    f1, f2 = project(D)
    r1 = dmm.solve_discrete(f1, w_h, w_v, T, n_iters, **dmm_kw)
    r2 = dmm.solve_discrete(f2, w_h, w_v, T, n_iters, **dmm_kw)
    u1, u2 = refine_flow(D, w_h, w_v, r1.labels, r2.labels, params)
    return FlowResult(f1=f1, f2=f2, layer1=r1, layer2=r2, u1=u1, u2=u2)
