"""Pins of the oracle's forward-mode derivatives: central finite differences of the plain
FP64 oracle (where both one-sided differences agree, i.e. no kink is crossed), and the
closed form of the zero-interaction case.  No GPU."""
import numpy as np
import pytest

import synth
from oracle import chain, dmm, grad, refine


def _fd(f, eps=1e-6):
    """(central, one-sided agreement mask) of a vector-valued f(t) at t = 0."""
    f0, fp, fm = f(0.0), f(eps), f(-eps)
    central = (fp - fm) / (2 * eps)
    right, left = (fp - f0) / eps, (f0 - fm) / eps
    smooth = np.abs(right - left) <= 1e-6 * np.maximum(1.0, np.abs(central))
    return central, smooth


@pytest.mark.parametrize("K,T", [(5, 1), (7, 2), (9, 3), (4, 10)])
def test_message_jvp_fd(K, T):
    g = np.random.default_rng(K + T)
    v, vd = g.normal(size=(6, K)), g.normal(size=(6, K))
    w, wd = g.random(6) + 0.1, g.normal(size=6)
    _, tan = grad.message_jvp(v, vd, w, wd, T)
    fd, ok = _fd(lambda t: chain.message(v + t * vd, w + t * wd, T))
    assert ok.mean() > 0.9
    np.testing.assert_allclose(tan[ok], fd[ok], atol=1e-6)


def test_min_marginals_zero_interaction_closed_form():
    """w = 0: d mbar_j = d a_j - d a_j(k*) (identity minus the argmin selection)."""
    g = np.random.default_rng(3)
    a, ad = g.random((2, 5, 6)), g.normal(size=(2, 5, 6))
    w = np.zeros((2, 4))
    mm, mmd = grad.min_marginals_jvp(a, ad, w, np.zeros_like(w), 2)
    k = np.argmin(a, axis=2)
    want = ad - np.take_along_axis(ad, k[..., None], axis=2)
    np.testing.assert_allclose(mmd, want, atol=1e-12)


@pytest.mark.parametrize("gammas", [(0.25, 0.25, 1.0), (1.0,)])
def test_iterative_minorant_jvp_fd(gammas):
    g = np.random.default_rng(11)
    a, ad = g.random((3, 7, 5)) * 2, g.normal(size=(3, 7, 5))
    w, wd = g.random((3, 6)) * 0.5, g.normal(size=(3, 6))
    _, hd = grad.iterative_minorant_jvp(a, ad, w, wd, 2, gammas)
    fd, ok = _fd(lambda t: chain.iterative_minorant(a + t * ad, w + t * wd, 2, gammas))
    assert ok.mean() > 0.9
    np.testing.assert_allclose(hd[ok], fd[ok], atol=2e-6)


@pytest.mark.parametrize("minorant", ["iterative", "naive"])
def test_solve_discrete_jvp_fd(minorant):
    theta, w_h, w_v = synth.tiny_instance(5, 6, 4, seed=13, w_max=0.5)
    theta = theta.astype(np.float64); w_h = w_h.astype(np.float64); w_v = w_v.astype(np.float64)
    g = np.random.default_rng(1)
    td, whd, wvd = g.normal(size=theta.shape), g.normal(size=w_h.shape), g.normal(size=w_v.shape)
    mm, mmd, lb, lbd, _ = grad.solve_discrete_jvp(theta, td, w_h, whd, w_v, wvd, 2, 3, minorant=minorant)

    def f(t):
        r = dmm.solve_discrete(theta + t * td, w_h + t * whd, w_v + t * wvd, 2, 3, minorant=minorant)
        return np.concatenate([r.minmarg.ravel(), [r.lower_bound]])
    fd, ok = _fd(f)
    got = np.concatenate([mmd.ravel(), [lbd]])
    assert ok.mean() > 0.9
    np.testing.assert_allclose(got[ok], fd[ok], atol=2e-6)
    assert ok[-1], "lower bound should be smooth at a generic point"


@pytest.mark.parametrize("warps,iters", [(1, 20), (3, 15)])
def test_refine_jvp_fd(warps, iters):
    theta, w_h, w_v = synth.tiny_instance(6, 7, 8, seed=warps, w_max=0.5)
    theta = theta.astype(np.float64); w_h = w_h.astype(np.float64); w_v = w_v.astype(np.float64)
    labels = np.random.default_rng(4).integers(1, 7, (6, 7))
    P = refine.RefineParams(C=2.0, n_warps=warps, n_iters=iters)
    g = np.random.default_rng(2)
    td, whd, wvd = g.normal(size=theta.shape), g.normal(size=w_h.shape), g.normal(size=w_v.shape)
    _, ud = grad.refine_continuous_jvp(theta, td, w_h, whd, w_v, wvd, labels, P)
    fd, ok = _fd(lambda t: refine.refine_continuous(theta + t * td, w_h + t * whd, w_v + t * wvd, labels, P))
    # after the first warp many pixels sit exactly on integer clamp bounds, where the
    # interpolated data term has a kink: only points with matching one-sided slopes count
    assert ok.mean() > (0.8 if warps == 1 else 0.4)
    np.testing.assert_allclose(ud[ok], fd[ok], atol=2e-6)
