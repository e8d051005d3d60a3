"""Continuous refinement by the non-linear primal-dual method (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Problem (Sec. 2.1, eq. mrf_formulation): min_u D(u) + R(Au) with
(Au)_e = u_i - u_j for every edge e = (i, j) of the 4-connected grid (j the
right or the lower neighbour), R(Au) = sum_e w_e r((Au)_e).

Difference-of-convex split (Sec. 2.4, eq. r-decompose):
    r = r_{eps,delta} - r_{0, C + delta - eps*delta},
    r_{alpha,beta}(t) = alpha |t|               if |t| <= beta
                      = |t| - beta (1 - alpha)  otherwise,
which for eps = 1, delta = 0 is r(t) = min(|t|, C).

Primal-dual form (Sec. 2.4, eq. cont_problem and the non-linear operator):
x = (u, q), y = (p, d = 1), A(x) = [Au ; -<Au, q>], G(x) = R_-^*(q) + D(u),
F^*(y) = R_+^*(p).  Valkonen's iteration (eq. cont_iterates) with
grad A(x)^T y = (A^T (p - q), -Au) reads, component by component,

    u+ = prox_{tau D~}( u - tau A^T (p - q) )
    q+ = prox_{tau R_-^*}( q + tau A u )
    p+ = prox_{sigma R_+^*}( p + sigma A (2 u+ - u) ).

The prox of (w r_{alpha,beta})^* at t* (eq. pprox): t' = t* if |t*| <= alpha w,
else max(alpha w, |t*| - beta sigma) sign(t*); then clamp to [-w, w].  R_-^*
uses alpha = 0, beta = C + delta - eps*delta with step tau (the paper gives
only the F^* case; this is the same formula for the other pair of constants).

Data term (Sec. 3.1): around the current point u0 ("u ring") D is replaced
by the convex piecewise-linear D~ with slopes s_L (left of u0) and s_R (right
of u0), restricted to [u0 - h, u0 + h]; the prox of tau D~ is a two-slope soft
threshold followed by the clamp.  Every ``n_iters`` iterations the data term
is linearised again at the current u ("warping").

Readings where the paper's text is garbled or silent:
  * slopes: s_L = (D(u0) - D(u0 - h)) / h, s_R = (D(u0 + h) - D(u0)) / h (the
    printed formulas are negatives of each other); if s_L > s_R both become
    their mean (the paper's convexification);
  * D between labels: linear interpolation of the cost volume along the
    label axis, with the argument clamped to [0, K-1]; at the ends of the
    label range the missing one-sided slope copies the other one;
  * prox of tau D~: hat u - tau s_R if hat u > u0 + tau s_R; hat u - tau s_L if
    hat u < u0 + tau s_L; u0 otherwise; then clamp to [u0 - h, u0 + h]
    intersected with [0, K-1];
  * p = q = 0 at the start, u = u0 = the discrete labels; p and q carry over
    between warps.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "RefineParams",
    "interp_cost",
    "linearize",
    "prox_data",
    "prox_conj",
    "grad_op",
    "grad_op_T",
    "refine_continuous",
    "r_penalty",
    "continuous_energy",
]


@dataclasses.dataclass
class RefineParams:
    C: float = 3.0
    eps: float = 1.0
    delta: float = 0.0
    h: float = 1.0
    tau: float = 0.3
    sigma: float = 0.3
    n_warps: int = 5
    n_iters: int = 40


def r_alpha_beta(t, alpha, beta):
    a = np.abs(t)
    return np.where(a <= beta, alpha * a, a - beta * (1.0 - alpha))


def r_penalty(t, C, eps, delta):
    """r = r_{eps,delta} - r_{0, C + delta - eps delta} (eq. r-decompose)."""
    return r_alpha_beta(t, eps, delta) - r_alpha_beta(t, 0.0, C + delta - eps * delta)


def interp_cost(theta, v):
    """D_i(v_i): linear interpolation of theta_i along the label axis at v_i (clamped)."""
    theta = np.asarray(theta, np.float64)
    H, W, K = theta.shape
    v = np.clip(np.asarray(v, np.float64), 0.0, K - 1.0)
    k0 = np.floor(v).astype(np.int64)
    k0 = np.minimum(k0, K - 1)
    k1 = np.minimum(k0 + 1, K - 1)
    t = v - k0
    d0 = np.take_along_axis(theta, k0[:, :, None], axis=2)[:, :, 0]
    d1 = np.take_along_axis(theta, k1[:, :, None], axis=2)[:, :, 0]
    return (1.0 - t) * d0 + t * d1


def linearize(theta, u0, h):
    """Slopes (s_L, s_R) of the convex two-slope model of D around u0 (Sec. 3.1)."""
    theta = np.asarray(theta, np.float64)
    K = theta.shape[2]
    u0 = np.asarray(u0, np.float64)
    Dc = interp_cost(theta, u0)
    Dm = interp_cost(theta, u0 - h)
    Dp = interp_cost(theta, u0 + h)
    sL = (Dc - Dm) / h
    sR = (Dp - Dc) / h
    has_left = u0 - h >= 0.0
    has_right = u0 + h <= K - 1.0
    sL = np.where(has_left, sL, np.where(has_right, sR, 0.0))
    sR = np.where(has_right, sR, np.where(has_left, sL, 0.0))
    mean = 0.5 * (sL + sR)
    nonconvex = sL > sR
    sL = np.where(nonconvex, mean, sL)
    sR = np.where(nonconvex, mean, sR)
    return sL, sR


def prox_data(u_hat, u0, sL, sR, tau, h, K):
    """prox of tau * D~ at u_hat: two-slope soft threshold, then the box clamp (Sec. 3.1)."""
    out = np.where(u_hat > u0 + tau * sR, u_hat - tau * sR,
                   np.where(u_hat < u0 + tau * sL, u_hat - tau * sL, u0))
    lo = np.maximum(u0 - h, 0.0)
    hi = np.minimum(u0 + h, K - 1.0)
    return np.clip(out, lo, hi)


def prox_conj(t_star, w, alpha, beta, step):
    """prox of step*(w r_{alpha,beta})^* at t_star (eq. pprox), component-wise."""
    a = np.abs(t_star)
    t = np.where(a <= alpha * w, t_star, np.maximum(alpha * w, a - beta * step) * np.sign(t_star))
    return np.clip(t, -w, w)


def grad_op(u):
    """(Au)_e = u_i - u_j for right (h) and lower (v) neighbours j of i."""
    gh = u[:, :-1] - u[:, 1:]
    gv = u[:-1, :] - u[1:, :]
    return gh, gv


def grad_op_T(yh, yv, shape):
    """Exact transpose of ``grad_op``."""
    H, W = shape
    out = np.zeros((H, W))
    out[:, :-1] += yh
    out[:, 1:] -= yh
    out[:-1, :] += yv
    out[1:, :] -= yv
    return out


def continuous_energy(theta, w_h, w_v, u, C, eps, delta):
    """E(u) = sum_i D_i(u_i) + sum_e w_e r((Au)_e) with interpolated D."""
    gh, gv = grad_op(np.asarray(u, np.float64))
    return float(interp_cost(theta, u).sum()
                 + (np.asarray(w_h, np.float64) * r_penalty(gh, C, eps, delta)).sum()
                 + (np.asarray(w_v, np.float64) * r_penalty(gv, C, eps, delta)).sum())


def refine_continuous(theta, w_h, w_v, labels, params: RefineParams, *, return_state: bool = False):
    """Warped non-linear primal-dual refinement starting from the discrete labels."""
    theta = np.asarray(theta, np.float64)
    H, W, K = theta.shape
    w_h = np.asarray(w_h, np.float64)
    w_v = np.asarray(w_v, np.float64)
    P = params
    beta_minus = P.C + P.delta - P.eps * P.delta
    u = np.asarray(labels, np.float64).copy()
    ph = np.zeros((H, W - 1)); pv = np.zeros((H - 1, W))
    qh = np.zeros((H, W - 1)); qv = np.zeros((H - 1, W))
    for _ in range(P.n_warps):
        u0 = u.copy()
        sL, sR = linearize(theta, u0, P.h)
        for _ in range(P.n_iters):
            u_hat = u - P.tau * grad_op_T(ph - qh, pv - qv, (H, W))
            u_new = prox_data(u_hat, u0, sL, sR, P.tau, P.h, K)
            gh, gv = grad_op(u)
            qh = prox_conj(qh + P.tau * gh, w_h, 0.0, beta_minus, P.tau)
            qv = prox_conj(qv + P.tau * gv, w_v, 0.0, beta_minus, P.tau)
            bh, bv = grad_op(2.0 * u_new - u)
            ph = prox_conj(ph + P.sigma * bh, w_h, P.eps, P.delta, P.sigma)
            pv = prox_conj(pv + P.sigma * bv, w_v, P.eps, P.delta, P.sigma)
            u = u_new
    if return_state:
        return u, dict(ph=ph, pv=pv, qh=qh, qv=qv)
    return u
