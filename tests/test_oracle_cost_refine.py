"""Pins of the oracle's cost volume and continuous refinement. No GPU."""
import numpy as np
import pytest

import synth
from oracle import cost_volume, refine, energy


def test_cost_volume_constant_shift_zero_at_true_disparity():
    """Noise-free integer shift d0: the SAD at d0 vanishes wherever the window sees valid pixels."""
    g = np.random.default_rng(0)
    H, W, K, d0 = 6, 20, 8, 3
    L = g.random((H, W))
    R = np.zeros_like(L)
    R[:, : W - d0] = L[:, d0:]          # I_R(x - d0) = I_L(x)
    R[:, W - d0:] = g.random((H, d0))
    th = cost_volume.sad_cost_volume(L, R, K)
    assert np.all(th[:, d0 + 1: W - 1, d0] == 0.0)
    assert th.max() <= 0.3 + 1e-15 and th.min() >= 0.0


def test_cost_volume_hand_example():
    """2x3 images, K = 2, 3x3 window with clamp-to-edge, hand-computed."""
    L = np.array([[0.1, 0.2, 0.4], [0.3, 0.3, 0.0]])
    R = np.array([[0.0, 0.2, 0.1], [0.1, 0.5, 0.2]])
    th = cost_volume.sad_cost_volume(L, R, 2, window=3, trunc=10.0)
    # d = 0: e = |L - R|
    e0 = np.abs(L - R)
    # pixel (0,0): window rows {0,0,1}, cols {0,0,1}
    want = (e0[[0, 0, 1]][:, [0, 0, 1]]).sum() / 9
    assert th[0, 0, 0] == pytest.approx(want)
    # d = 1: e(x) = |L(x) - R(x-1)| for x >= 1, else trunc
    e1 = np.full((2, 3), 10.0)
    e1[:, 1:] = np.abs(L[:, 1:] - R[:, :-1])
    want = (e1[[0, 1, 1]][:, [1, 2, 2]]).sum() / 9
    assert th[1, 2, 1] == pytest.approx(want)


def test_contrast_weights_hand_example():
    L = np.array([[0.0, 0.1, 0.1], [0.5, 0.1, 0.1]])
    w_h, w_v = cost_volume.contrast_weights(L, lambda_pw=0.1, sigma_c=0.1)
    assert w_h[0, 0] == pytest.approx(0.1 * np.exp(-1.0))
    assert w_h[0, 1] == pytest.approx(0.1)
    assert w_v[0, 0] == pytest.approx(0.1 * np.exp(-5.0))


def test_half_rounding_bound():
    x = np.random.default_rng(1).random(10000) * 0.3
    r = cost_volume.round_half(x)
    normal = np.abs(x) >= 2.0 ** -14
    assert np.all(np.abs(r - x)[normal] <= np.abs(x)[normal] * 2.0 ** -11)
    assert np.all(np.abs(r - x)[~normal] <= 2.0 ** -25)


# ---------------------------------------------------------------- refinement prox maps

def test_prox_data_matches_1d_minimisation():
    """Two-slope soft threshold + clamp is the prox of tau*D~ (Sec. 3.1), checked on a fine grid."""
    g = np.random.default_rng(2)
    K, h, tau = 10, 1.0, 0.3
    for _ in range(200):
        u0 = g.uniform(0, K - 1)
        sL, sR = np.sort(g.normal(size=2) * 2)
        uh = u0 + g.normal() * 1.5
        lo, hi = max(u0 - h, 0.0), min(u0 + h, K - 1.0)
        grid = np.linspace(lo, hi, 200001)
        obj = 0.5 * (grid - uh) ** 2 + tau * np.where(grid <= u0, sL * (grid - u0), sR * (grid - u0))
        want = grid[np.argmin(obj)]
        got = refine.prox_data(np.array([uh]), np.array([u0]), np.array([sL]), np.array([sR]), tau, h, K)[0]
        assert got == pytest.approx(want, abs=2e-5)


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.0, 3.0), (0.5, 0.7), (0.2, 2.0)])
def test_prox_conj_matches_numeric_conjugate(alpha, beta):
    """eq. pprox against prox of the numerically conjugated w r_{alpha,beta} (reads the domain as |t*| <= w)."""
    g = np.random.default_rng(int(alpha * 10 + beta * 100))
    w, step = 0.7, 0.3
    t = np.linspace(-60, 60, 240001)
    f = w * refine.r_alpha_beta(t, alpha, beta)
    s_grid = np.linspace(-w, w, 4001)
    fstar = np.max(s_grid[:, None] * t[None, :] - f[None, :], axis=1)
    for _ in range(40):
        ts = g.normal() * 1.2
        obj = fstar + (s_grid - ts) ** 2 / (2 * step)
        want = s_grid[np.argmin(obj)]
        got = refine.prox_conj(np.array([ts]), w, alpha, beta, step)[0]
        assert got == pytest.approx(want, abs=1e-3)


def test_r_decomposition_gives_truncated_linear():
    t = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(refine.r_penalty(t, 3.0, 1.0, 0.0), np.minimum(np.abs(t), 3.0), atol=1e-12)


def test_continuous_energy_equals_discrete_at_labels():
    """eps = 1, delta = 0, C = T: the continuous energy at integer u is the discrete energy (Sec. 2)."""
    theta, w_h, w_v = synth.tiny_instance(4, 5, 6, seed=3)
    x = np.random.default_rng(0).integers(0, 6, (4, 5))
    ec = refine.continuous_energy(theta, w_h, w_v, x.astype(float), 2.0, 1.0, 0.0)
    assert ec == pytest.approx(energy.grid_energy(theta, w_h, w_v, 2, x), abs=1e-12)


def test_linearize_at_integer_labels():
    theta, _, _ = synth.tiny_instance(2, 3, 5, seed=1)
    u0 = np.array([[0, 2, 4], [1, 3, 2]], dtype=float)
    sL, sR = refine.linearize(theta, u0, 1.0)
    th = theta.astype(np.float64)
    for y in range(2):
        for x in range(3):
            k = int(u0[y, x])
            l = th[y, x, k] - th[y, x, k - 1] if k > 0 else None
            r = th[y, x, k + 1] - th[y, x, k] if k < 4 else None
            l = r if l is None else l
            r = l if r is None else r
            if l > r:
                l = r = 0.5 * (l + r)
            assert sL[y, x] == pytest.approx(l) and sR[y, x] == pytest.approx(r)


def test_zero_weights_closed_form():
    """w = 0 decouples pixels: u moves to the minimiser of D~ on the box (prox fixed point)."""
    theta, w_h, w_v = synth.tiny_instance(3, 4, 6, seed=5)
    w_h[:] = 0.0
    w_v[:] = 0.0
    labels = np.random.default_rng(1).integers(0, 6, (3, 4))
    P = refine.RefineParams(C=2.0, n_warps=1, n_iters=200)
    u = refine.refine_continuous(theta, w_h, w_v, labels, P)
    sL, sR = refine.linearize(theta, labels.astype(float), 1.0)
    u0 = labels.astype(float)
    want = np.where(sL > 0, np.maximum(u0 - 1, 0), np.where(sR < 0, np.minimum(u0 + 1, 5), u0))
    np.testing.assert_allclose(u, want, atol=1e-9)


def test_convex_case_reaches_lp_optimum():
    """C -> infinity (q stays 0): plain TV + piecewise-linear data; PDHG reaches the LP optimum."""
    from scipy.optimize import linprog
    theta, w_h, w_v = synth.tiny_instance(4, 4, 6, seed=9, w_max=0.5)
    labels = np.random.default_rng(3).integers(1, 5, (4, 4))
    P = refine.RefineParams(C=1e9, n_warps=1, n_iters=6000)
    u = refine.refine_continuous(theta, w_h, w_v, labels, P)
    u0 = labels.astype(float)
    sL, sR = refine.linearize(theta, u0, 1.0)
    H, W = 4, 4
    n = H * W
    eh = [(y * W + x, y * W + x + 1, w_h[y, x]) for y in range(H) for x in range(W - 1)]
    ev = [(y * W + x, (y + 1) * W + x, w_v[y, x]) for y in range(H - 1) for x in range(W)]
    edges = eh + ev
    m = len(edges)
    # variables: u (n), a+ (n), a- (n), t (m); D~ = sR a+ - sL a-, u - u0 = a+ - a-
    nvar = 3 * n + m
    c = np.concatenate([np.zeros(n), sR.reshape(-1), -sL.reshape(-1), np.array([e[2] for e in edges])])
    A_eq = np.zeros((n, nvar)); b_eq = u0.reshape(-1).copy()
    for i in range(n):
        A_eq[i, i] = 1; A_eq[i, n + i] = -1; A_eq[i, 2 * n + i] = 1
    A_ub = np.zeros((2 * m, nvar)); b_ub = np.zeros(2 * m)
    for k, (i, j, _) in enumerate(edges):
        A_ub[2 * k, i] = 1; A_ub[2 * k, j] = -1; A_ub[2 * k, 3 * n + k] = -1
        A_ub[2 * k + 1, i] = -1; A_ub[2 * k + 1, j] = 1; A_ub[2 * k + 1, 3 * n + k] = -1
    lo = np.maximum(u0 - 1, 0).reshape(-1); hi = np.minimum(u0 + 1, 5).reshape(-1)
    bounds = [(lo[i], hi[i]) for i in range(n)] + [(0, None)] * (2 * n) + [(0, None)] * m
    lp = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq, bounds=bounds, method="highs")
    assert lp.status == 0

    def obj(uu):
        d = uu - u0
        data = np.where(d <= 0, sL * d, sR * d).sum()
        gh, gv = refine.grad_op(uu)
        return data + (w_h * np.abs(gh)).sum() + (w_v * np.abs(gv)).sum()
    assert obj(u) == pytest.approx(lp.fun, abs=1e-4)
