"""Forward-mode (dual-number) derivatives through the oracle, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Every function here carries a pair (value, tangent) through the same steps as
the corresponding oracle function (chain.py, dmm.py, refine.py), in the same
order.  Minimisations pass on the tangent of the selected candidate (the
lowest-index candidate on exact ties), clamps and soft thresholds pass on the
tangent of the active branch: the result is the directional derivative of the
piecewise-linear map wherever the branch choices are locally constant.  This is
a different algorithm from the GPU's reverse-mode adjoint; the two meet only
through <grad, direction>.  Central finite differences of the plain oracle pin
these functions (tests/test_oracle_grad.py).
"""
from __future__ import annotations

import numpy as np

from . import chain
from .refine import RefineParams, r_alpha_beta  # noqa: F401  (r_alpha_beta kept for symmetry of imports)

__all__ = [
    "message_jvp",
    "min_marginals_jvp",
    "iterative_minorant_jvp",
    "naive_minorant_jvp",
    "solve_discrete_jvp",
    "refine_continuous_jvp",
]


def _take(x, idx):
    return np.take_along_axis(x, idx[:, None], axis=1)[:, 0]


def message_jvp(v, vd, w, wd, T):
    """phi(b) = min( min_{|a-b|<T} v(a) + w|a-b| , min_a v(a) + wT ) with its tangent."""
    v = np.asarray(v, np.float64)
    C, K = v.shape
    w = np.asarray(w, np.float64)[:, None]
    wd = np.asarray(wd, np.float64)[:, None]
    amin = np.argmin(v, axis=1)
    best = (_take(v, amin)[:, None] + w * T) * np.ones((1, K))
    bestd = (_take(vd, amin)[:, None] + wd * T) * np.ones((1, K))
    # window candidates in order d = 0, -1, +1, -2, +2, ... ; strict improvement keeps the earlier one
    order = [0]
    for k in range(1, T):
        order += [-k, k]
    cand_best = np.full((C, K), np.inf)
    cand_bestd = np.zeros((C, K))
    for d in order:
        if abs(d) >= K:
            continue
        val = np.full((C, K), np.inf)
        dot = np.zeros((C, K))
        if d >= 0:
            val[:, : K - d] = v[:, d:]
            dot[:, : K - d] = vd[:, d:]
        else:
            val[:, -d:] = v[:, : K + d]
            dot[:, -d:] = vd[:, : K + d]
        val = val + w * abs(d)
        dot = dot + wd * abs(d)
        better = val < cand_best
        cand_best = np.where(better, val, cand_best)
        cand_bestd = np.where(better, dot, cand_bestd)
    use_window = cand_best <= best
    return np.where(use_window, cand_best, best), np.where(use_window, cand_bestd, bestd)


def _normalize_jvp(m, md):
    k = np.argmin(m, axis=-1)
    mn = np.take_along_axis(m, k[..., None], axis=-1)
    mnd = np.take_along_axis(md, k[..., None], axis=-1)
    return m - mn, md - mnd


def min_marginals_jvp(a, ad, w, wd, T, normalized=True):
    a = np.asarray(a, np.float64)
    C, n, K = a.shape
    L = np.zeros((C, n, K)); Ld = np.zeros((C, n, K))
    R = np.zeros((C, n, K)); Rd = np.zeros((C, n, K))
    for j in range(1, n):
        L[:, j], Ld[:, j] = message_jvp(L[:, j - 1] + a[:, j - 1], Ld[:, j - 1] + ad[:, j - 1], w[:, j - 1],
                                        wd[:, j - 1], T)
    for j in range(n - 2, -1, -1):
        R[:, j], Rd[:, j] = message_jvp(R[:, j + 1] + a[:, j + 1], Rd[:, j + 1] + ad[:, j + 1], w[:, j], wd[:, j], T)
    m = a + L + R
    md = ad + Ld + Rd
    if normalized:
        return _normalize_jvp(m, md)
    return m, md


def iterative_minorant_jvp(a, ad, w, wd, T, gammas):
    """Same steps as chain.iterative_minorant, with tangents."""
    a = np.asarray(a, np.float64)
    C, n, K = a.shape
    r = a.copy(); rd = np.array(ad, np.float64, copy=True)
    h = np.zeros_like(r); hd = np.zeros_like(r)
    L = np.zeros((C, n, K)); Ld = np.zeros((C, n, K))
    R = np.zeros((C, n, K)); Rd = np.zeros((C, n, K))
    for j in range(n - 2, -1, -1):
        R[:, j], Rd[:, j] = message_jvp(R[:, j + 1] + r[:, j + 1], Rd[:, j + 1] + rd[:, j + 1], w[:, j], wd[:, j], T)
    for s, g in enumerate(gammas):
        order = range(n) if s % 2 == 0 else range(n - 1, -1, -1)
        for j in order:
            m = r[:, j] + L[:, j] + R[:, j]
            md = rd[:, j] + Ld[:, j] + Rd[:, j]
            mn, mnd = _normalize_jvp(m, md)
            d, dd = g * mn, g * mnd
            r[:, j] -= d; rd[:, j] -= dd
            h[:, j] += d; hd[:, j] += dd
            if s % 2 == 0 and j + 1 < n:
                L[:, j + 1], Ld[:, j + 1] = message_jvp(L[:, j] + r[:, j], Ld[:, j] + rd[:, j], w[:, j], wd[:, j], T)
            if s % 2 == 1 and j - 1 >= 0:
                R[:, j - 1], Rd[:, j - 1] = message_jvp(R[:, j] + r[:, j], Rd[:, j] + rd[:, j], w[:, j - 1],
                                                        wd[:, j - 1], T)
    return h, hd


def naive_minorant_jvp(a, ad, w, wd, T):
    n = np.asarray(a).shape[1]
    m, md = min_marginals_jvp(a, ad, w, wd, T, normalized=True)
    return m / float(n), md / float(n)


def _cols(x):
    return np.ascontiguousarray(np.transpose(x, (1, 0, 2)))


def _chain_opt_jvp(a, ad, w, wd, T):
    m, md = min_marginals_jvp(a, ad, w, wd, T, normalized=False)
    k = np.argmin(m[:, 0, :], axis=1)
    return _take(m[:, 0, :], k), _take(md[:, 0, :], k)


def solve_discrete_jvp(theta, thetad, w_h, w_hd, w_v, w_vd, T, n_iters, *, minorant="iterative",
                       gammas=(0.25, 0.25, 1.0), n_half_steps=None):
    """Tangents of Dual_MM's outputs (normalized row min-marginals, lower bound) for a
    direction (thetad, w_hd, w_vd).  Returns (minmarg, minmarg_dot, lb, lb_dot, labels)."""
    theta = np.asarray(theta, np.float64)
    thetad = np.asarray(thetad, np.float64)
    w_h = np.asarray(w_h, np.float64); w_hd = np.asarray(w_hd, np.float64)
    w_v = np.asarray(w_v, np.float64); w_vd = np.asarray(w_vd, np.float64)
    lam = np.zeros_like(theta); lamd = np.zeros_like(theta)
    steps = 2 * n_iters if n_half_steps is None else n_half_steps

    def minor(a, ad, w, wd):
        if minorant == "iterative":
            return iterative_minorant_jvp(a, ad, w, wd, T, gammas)
        return naive_minorant_jvp(a, ad, w, wd, T)

    for s in range(steps):
        if s % 2 == 0:
            h, hd = minor(theta - lam, thetad - lamd, w_h, w_hd)
            lam = lam + h; lamd = lamd + hd
        else:
            h, hd = minor(_cols(lam), _cols(lamd), w_v.T, w_vd.T)
            lam = lam - _cols(h); lamd = lamd - _cols(hd)
    mm, mmd = min_marginals_jvp(theta - lam, thetad - lamd, w_h, w_hd, T, normalized=True)
    labels = np.argmin(mm, axis=2)
    ro, rod = _chain_opt_jvp(theta - lam, thetad - lamd, w_h, w_hd, T)
    co, cod = _chain_opt_jvp(_cols(lam), _cols(lamd), w_v.T, w_vd.T, T)
    return mm, mmd, float(ro.sum() + co.sum()), float(rod.sum() + cod.sum()), labels


# ---------------------------------------------------------------------- refinement

def _interp_jvp(theta, thetad, v, vd):
    H, W, K = theta.shape
    inside = (v >= 0.0) & (v <= K - 1.0)
    vc = np.clip(v, 0.0, K - 1.0)
    vcd = np.where(inside, vd, 0.0)
    k0 = np.minimum(np.floor(vc).astype(np.int64), K - 1)
    k1 = np.minimum(k0 + 1, K - 1)
    t = vc - k0
    td = vcd
    d0 = np.take_along_axis(theta, k0[:, :, None], axis=2)[:, :, 0]
    d1 = np.take_along_axis(theta, k1[:, :, None], axis=2)[:, :, 0]
    d0d = np.take_along_axis(thetad, k0[:, :, None], axis=2)[:, :, 0]
    d1d = np.take_along_axis(thetad, k1[:, :, None], axis=2)[:, :, 0]
    val = (1.0 - t) * d0 + t * d1
    dot = (1.0 - t) * d0d + t * d1d + td * (d1 - d0)
    return val, dot


def _linearize_jvp(theta, thetad, u0, u0d, h):
    K = theta.shape[2]
    Dc, Dcd = _interp_jvp(theta, thetad, u0, u0d)
    Dm, Dmd = _interp_jvp(theta, thetad, u0 - h, u0d)
    Dp, Dpd = _interp_jvp(theta, thetad, u0 + h, u0d)
    sL, sLd = (Dc - Dm) / h, (Dcd - Dmd) / h
    sR, sRd = (Dp - Dc) / h, (Dpd - Dcd) / h
    has_l = u0 - h >= 0.0
    has_r = u0 + h <= K - 1.0
    sL2 = np.where(has_l, sL, np.where(has_r, sR, 0.0))
    sL2d = np.where(has_l, sLd, np.where(has_r, sRd, 0.0))
    sR2 = np.where(has_r, sR, np.where(has_l, sL, 0.0))
    sR2d = np.where(has_r, sRd, np.where(has_l, sLd, 0.0))
    nonconvex = sL2 > sR2
    mean, meand = 0.5 * (sL2 + sR2), 0.5 * (sL2d + sR2d)
    return (np.where(nonconvex, mean, sL2), np.where(nonconvex, meand, sL2d),
            np.where(nonconvex, mean, sR2), np.where(nonconvex, meand, sR2d))


def _prox_data_jvp(uh, uhd, u0, u0d, sL, sLd, sR, sRd, tau, h, K):
    zr = uh > u0 + tau * sR
    zl = (~zr) & (uh < u0 + tau * sL)
    v = np.where(zr, uh - tau * sR, np.where(zl, uh - tau * sL, u0))
    vd = np.where(zr, uhd - tau * sRd, np.where(zl, uhd - tau * sLd, u0d))
    lo_is_box = u0 - h >= 0.0
    lo = np.maximum(u0 - h, 0.0)
    lod = np.where(lo_is_box, u0d, 0.0)
    hi_is_box = u0 + h <= K - 1.0
    hi = np.minimum(u0 + h, K - 1.0)
    hid = np.where(hi_is_box, u0d, 0.0)
    below = v < lo
    above = (~below) & (v > hi)
    return (np.where(below, lo, np.where(above, hi, v)), np.where(below, lod, np.where(above, hid, vd)))


def _prox_conj_jvp(t, td, w, wd, alpha, beta, step):
    a = np.abs(t)
    sg = np.sign(t)
    inner = a <= alpha * w
    shrink = a - beta * step
    flat = (~inner) & (shrink < alpha * w)
    r = np.where(inner, t, np.where(flat, alpha * w * sg, shrink * sg))
    rd = np.where(inner, td, np.where(flat, alpha * wd * sg, td))
    below = r < -w
    above = (~below) & (r > w)
    return np.where(below, -w, np.where(above, w, r)), np.where(below, -wd, np.where(above, wd, rd))


def _grad_op(u):
    return u[:, :-1] - u[:, 1:], u[:-1, :] - u[1:, :]


def _grad_op_T(yh, yv, shape):
    H, W = shape
    out = np.zeros((H, W))
    out[:, :-1] += yh
    out[:, 1:] -= yh
    out[:-1, :] += yv
    out[1:, :] -= yv
    return out


def refine_continuous_jvp(theta, thetad, w_h, w_hd, w_v, w_vd, labels, P: RefineParams):
    """Tangent of the refined u for a direction (thetad, w_hd, w_vd); labels are constant."""
    theta = np.asarray(theta, np.float64)
    thetad = np.asarray(thetad, np.float64)
    H, W, K = theta.shape
    w_h = np.asarray(w_h, np.float64); w_hd = np.asarray(w_hd, np.float64)
    w_v = np.asarray(w_v, np.float64); w_vd = np.asarray(w_vd, np.float64)
    bm = P.C + P.delta - P.eps * P.delta
    u = np.asarray(labels, np.float64).copy(); ud = np.zeros((H, W))
    ph = np.zeros((H, W - 1)); phd = np.zeros_like(ph)
    pv = np.zeros((H - 1, W)); pvd = np.zeros_like(pv)
    qh = np.zeros((H, W - 1)); qhd = np.zeros_like(qh)
    qv = np.zeros((H - 1, W)); qvd = np.zeros_like(qv)
    for _ in range(P.n_warps):
        u0, u0d = u.copy(), ud.copy()
        sL, sLd, sR, sRd = _linearize_jvp(theta, thetad, u0, u0d, P.h)
        for _ in range(P.n_iters):
            uh = u - P.tau * _grad_op_T(ph - qh, pv - qv, (H, W))
            uhd = ud - P.tau * _grad_op_T(phd - qhd, pvd - qvd, (H, W))
            un, und = _prox_data_jvp(uh, uhd, u0, u0d, sL, sLd, sR, sRd, P.tau, P.h, K)
            gh, gv = _grad_op(u)
            ghd, gvd = _grad_op(ud)
            qh, qhd = _prox_conj_jvp(qh + P.tau * gh, qhd + P.tau * ghd, w_h, w_hd, 0.0, bm, P.tau)
            qv, qvd = _prox_conj_jvp(qv + P.tau * gv, qvd + P.tau * gvd, w_v, w_vd, 0.0, bm, P.tau)
            bh, bv = _grad_op(2.0 * un - u)
            bhd, bvd = _grad_op(2.0 * und - ud)
            ph, phd = _prox_conj_jvp(ph + P.sigma * bh, phd + P.sigma * bhd, w_h, w_hd, P.eps, P.delta, P.sigma)
            pv, pvd = _prox_conj_jvp(pv + P.sigma * bv, pvd + P.sigma * bvd, w_v, w_vd, P.eps, P.delta, P.sigma)
            u, ud = un, und
    return u, ud
