"""Pins of the optical-flow oracle (Sec. 2.2 "Flow", Sec. 3.2): the two-dimensional SAD cost,
the decoupled costs, the quadratic fit, its prox, and the refinement.  No GPU."""
import itertools

import numpy as np
import pytest

import synth
from oracle import cost_volume, dmm, energy, flow
from oracle.refine import RefineParams, grad_op, grad_op_T
from tests.mutation import mutated


def test_flow_cost_volume_reduces_to_stereo():
    """With one vertical label (K2 = 1, off2 = 0) and horizontal displacements -d the flow
    cost is the stereo SAD cost volume of the same pair: D[.][.][0][off1 - d] = theta[.][.][d]."""
    pair = synth.stereo_pair(23, 11, 6, seed=3)
    K = 6
    D = flow.flow_cost_volume(pair.left, pair.right, K, 1, K - 1, 0)
    th = cost_volume.sad_cost_volume(pair.left, pair.right, K)
    for d in range(K):
        np.testing.assert_array_equal(D[:, :, 0, K - 1 - d], th[:, :, d])


def test_flow_cost_volume_true_shift():
    """A noise-free integer displacement (d1, d2) = (2, -1): zero cost at its label wherever
    every window position's match lies inside the second image."""
    g = np.random.default_rng(0)
    H, W, d1, d2 = 9, 12, 2, -1
    A = g.random((H, W))
    B = g.random((H, W))
    for y in range(H):
        for x in range(W):
            if 0 <= y + d2 < H and 0 <= x + d1 < W:
                B[y + d2, x + d1] = A[y, x]
    D = flow.flow_cost_volume(A, B, 5, 5, 2, 2)
    i, j = d1 + 2, d2 + 2
    # interior: the window (clamped) and its displaced positions stay in the image
    assert np.all(D[2:H - 1, 1:W - 3, j, i] == 0.0)
    assert D[:, :, j, i].max() > 0.0           # near the borders the match leaves the image
    assert D.max() <= 0.3 + 1e-15 and D.min() >= 0.0


def test_flow_cost_volume_row_band():
    """A band of output rows equals the same rows of the whole volume."""
    pair = synth.flow_pair(17, 9, 2.0, seed=8)
    full = flow.flow_cost_volume(pair.first, pair.second, 5, 4, 2, 1)
    for lo, hi in [(0, 1), (3, 6), (8, 9), (0, 9)]:
        np.testing.assert_array_equal(flow.flow_cost_volume(pair.first, pair.second, 5, 4, 2, 1, rows=(lo, hi)),
                                      full[lo:hi])


def test_flow_cost_volume_hand_example():
    """2 x 3 images, one label pair, 3 x 3 clamped window, by hand."""
    A = np.array([[0.1, 0.2, 0.4], [0.3, 0.3, 0.0]])
    B = np.array([[0.0, 0.2, 0.1], [0.1, 0.5, 0.2]])
    D = flow.flow_cost_volume(A, B, 2, 2, 0, 1, trunc=10.0)   # label (i, j) = (1, 0): displacement (1, -1)
    e = np.full((2, 3), 10.0)
    e[1, 0] = abs(A[1, 0] - B[0, 1])
    e[1, 1] = abs(A[1, 1] - B[0, 2])
    # pixel (x=1, y=1): window rows {0, 1, 1}, columns {0, 1, 2}
    want = e[[0, 1, 1]][:, [0, 1, 2]].sum() / 9
    assert D[1, 1, 0, 1] == pytest.approx(want)


def test_project_by_definition():
    g = np.random.default_rng(1)
    D = g.random((3, 4, 5, 6))
    f1, f2 = flow.project(D)
    for y, x in itertools.product(range(3), range(4)):
        for a in range(6):
            assert f1[y, x, a] == min(D[y, x, b, a] for b in range(5))
        for b in range(5):
            assert f2[y, x, b] == min(D[y, x, b, a] for a in range(6))
    # optimistic: below every entry of its row / column of the table
    assert np.all(f1[:, :, None, :] <= D) and np.all(f2[:, :, :, None] <= D)


def test_single_pixel_layers_recover_the_joint_minimiser():
    """One pixel, no edges: each layer's labeling is the component of the joint argmin."""
    g = np.random.default_rng(2)
    for _ in range(5):
        D = g.random((1, 1, 4, 7))
        r = flow.solve_flow(D, np.zeros((1, 0)), np.zeros((0, 1)), 2, 1,
                            RefineParams(C=2.0, n_warps=0, n_iters=0))
        b, a = np.unravel_index(np.argmin(D[0, 0]), D[0, 0].shape)
        assert r.layer1.labels[0, 0] == a and r.layer2.labels[0, 0] == b


def test_interp2():
    g = np.random.default_rng(3)
    D = g.random((2, 2, 4, 5))
    yy, xx = np.meshgrid(range(2), range(2), indexing="ij")
    for a, b in [(0, 0), (4, 3), (2, 1)]:
        np.testing.assert_array_equal(flow.interp2(D, np.full((2, 2), float(a)), np.full((2, 2), float(b))),
                                      D[:, :, b, a])
    v = flow.interp2(D, np.full((2, 2), 1.25), np.full((2, 2), 2.5))
    want = 0.5 * (0.75 * D[:, :, 2, 1] + 0.25 * D[:, :, 2, 2]) + 0.5 * (0.75 * D[:, :, 3, 1] + 0.25 * D[:, :, 3, 2])
    np.testing.assert_allclose(v, want, atol=1e-15)
    # arguments beyond the label range are clamped
    np.testing.assert_array_equal(flow.interp2(D, np.full((2, 2), -3.0), np.full((2, 2), 9.0)), D[:, :, 3, 0])


def test_quadfit_is_exact_for_a_separable_quadratic():
    """A table sampled from c + g.(u - m) + (a1 (u1 - m1)^2 + a2 (u2 - m2)^2) / 2 with a1, a2 > 0:
    central differences are exact, so L and Q are the gradient and the Hessian's diagonal."""
    K1, K2 = 7, 6
    x1, x2 = np.meshgrid(np.arange(K1), np.arange(K2))
    a1, a2, m1, m2 = 0.5, 1.5, 2.3, 3.7
    tab = 1.0 + 0.5 * a1 * (x1 - m1) ** 2 + 0.5 * a2 * (x2 - m2) ** 2
    D = np.broadcast_to(tab, (2, 3, K2, K1)).copy()
    u1 = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 2.0]])
    u2 = np.array([[1.0, 2.0, 3.0], [4.0, 2.0, 1.0]])
    L1, L2, Q1, Q2 = flow.linearize_quadfit(D, u1, u2, 1.0)
    np.testing.assert_allclose(L1, a1 * (u1 - m1), atol=1e-12)
    np.testing.assert_allclose(L2, a2 * (u2 - m2), atol=1e-12)
    np.testing.assert_allclose(Q1, a1, atol=1e-12)
    np.testing.assert_allclose(Q2, a2, atol=1e-12)


def test_quadfit_keeps_the_psd_part():
    """Negative curvature is dropped (Q = 0), positive kept."""
    D = np.zeros((1, 1, 3, 3))
    D[0, 0, 1, :] = [1.0, 2.0, 1.0]      # along x1 at x2 = 1: concave
    D[0, 0, :, 1] = [4.0, 2.0, 3.0]      # along x2 at x1 = 1: convex, second difference 3
    L1, L2, Q1, Q2 = flow.linearize_quadfit(D, np.ones((1, 1)), np.ones((1, 1)), 1.0)
    assert Q1[0, 0] == 0.0 and Q2[0, 0] == 3.0
    assert L1[0, 0] == 0.0 and L2[0, 0] == pytest.approx(-0.5)


def _prox_objective(v, u_hat, u0, L, Q, tau):
    return 0.5 * (v - u_hat) ** 2 + tau * (L * (v - u0) + 0.5 * Q * (v - u0) ** 2)


@pytest.mark.parametrize("seed", range(5))
def test_prox_flow_matches_2d_minimisation(seed):
    """eq. prox_flow against brute-force minimisation of the two-component prox objective
    (quadratic model + box) on a fine grid."""
    g = np.random.default_rng(seed)
    K, h, tau = 10, 1.0, 0.3
    for _ in range(6):
        u0 = g.integers(0, K, 2).astype(np.float64)
        u_hat = u0 + g.normal(0, 1.5, 2)
        L = g.normal(0, 2.0, 2)
        Q = np.maximum(g.normal(1.0, 1.5, 2), 0.0)
        got = np.array([flow.prox_flow(u_hat[k], u0[k], L[k], Q[k], tau, h, K) for k in range(2)])
        grids = [np.linspace(max(u0[k] - h, 0.0), min(u0[k] + h, K - 1.0), 801) for k in range(2)]
        V1, V2 = np.meshgrid(*grids, indexing="ij")
        obj = _prox_objective(V1, u_hat[0], u0[0], L[0], Q[0], tau) + _prox_objective(V2, u_hat[1], u0[1], L[1],
                                                                                       Q[1], tau)
        i = np.unravel_index(np.argmin(obj), obj.shape)
        np.testing.assert_allclose(got, [V1[i], V2[i]], atol=3e-3)


def test_prox_flow_printed_denominator_fails_the_minimisation():
    """The printed denominator 1 + tau L (taken literally) does not minimise the prox
    objective: the reading 1 + tau Q is the one that does."""
    mut = mutated(flow, ("v = (u_hat + tau * (Q * u0 - L)) / (1.0 + tau * Q)",
                         "v = (u_hat + tau * (Q * u0 - L)) / (1.0 + tau * L)"))
    g = np.random.default_rng(7)
    worst = 0.0
    for _ in range(50):
        u0 = float(g.integers(1, 9))
        u_hat, L, Q = u0 + g.normal(0, 0.5), g.normal(0, 2.0), abs(g.normal(1.0, 1.0))
        grid = np.linspace(u0 - 1.0, u0 + 1.0, 20001)
        best = grid[np.argmin(_prox_objective(grid, u_hat, u0, L, Q, 0.3))]
        worst = max(worst, abs(float(mut.prox_flow(u_hat, u0, L, Q, 0.3, 1.0, 10)) - best))
    assert worst > 0.05


def test_refine_flow_zero_weights_reaches_the_model_minimiser():
    """w = 0: each pixel and component minimises its own quadratic model on the box."""
    g = np.random.default_rng(4)
    H, W, K1, K2 = 4, 5, 8, 6
    D = g.random((H, W, K2, K1))
    l1 = g.integers(1, K1 - 1, (H, W))
    l2 = g.integers(1, K2 - 1, (H, W))
    P = RefineParams(C=2.0, tau=0.3, sigma=0.3, n_warps=1, n_iters=3000)
    u1, u2 = flow.refine_flow(D, np.zeros((H, W - 1)), np.zeros((H - 1, W)), l1, l2, P)
    L1, L2, Q1, Q2 = flow.linearize_quadfit(D, l1.astype(float), l2.astype(float), 1.0)
    for u, l, L, Q, K in ((u1, l1, L1, Q1, K1), (u2, l2, L2, Q2, K2)):
        lo, hi = np.maximum(l - 1.0, 0.0), np.minimum(l + 1.0, K - 1.0)
        want = np.where(Q > 0, np.clip(l - L / np.where(Q > 0, Q, 1.0), lo, hi),
                        np.where(L > 0, lo, np.where(L < 0, hi, l)))
        np.testing.assert_allclose(u, want, atol=1e-6)


def _flow_step_instance(seed):
    """3 x 4 grid with two flat halves far apart in both components (edges across the step
    keep |Au| > C), convex quadratic tables with random curvatures, weights U[0.2, 0.6]."""
    g = np.random.default_rng(seed)
    H, W, K1, K2 = 3, 4, 12, 10
    x1 = np.where(np.arange(W)[None, :] < 2, 2, 8) + g.integers(0, 2, (H, W))
    x2 = np.where(np.arange(W)[None, :] < 2, 6, 1) + g.integers(0, 2, (H, W))
    a1 = g.uniform(0.02, 0.2, (H, W, 1, 1))
    a2 = g.uniform(0.02, 0.2, (H, W, 1, 1))
    k1 = np.arange(K1)[None, None, None, :]
    k2 = np.arange(K2)[None, None, :, None]
    D = a1 * (k1 - x1[:, :, None, None] - 0.3) ** 2 + a2 * (k2 - x2[:, :, None, None] + 0.2) ** 2
    return D, g.uniform(0.2, 0.6, (H, W - 1)), g.uniform(0.2, 0.6, (H - 1, W)), x1, x2


@pytest.mark.parametrize("seed", [0, 1])
def test_refine_flow_fixed_point_is_critical(seed):
    """Non-convex regulariser (C = 2): the fixed point of the iteration satisfies, per
    component, p in dR_+(Au), q in dR_-(Au), -A^T(p - q) = grad D~(u) + normal cone of the box."""
    D, w_h, w_v, x1, x2 = _flow_step_instance(seed)
    P = RefineParams(C=2.0, tau=0.25, sigma=0.25, n_warps=1, n_iters=2500)
    u1, u2, st = flow.refine_flow(D, w_h, w_v, x1, x2, P, return_state=True)
    L1, L2, Q1, Q2 = flow.linearize_quadfit(D, x1.astype(float), x2.astype(float), 1.0)
    tol = 1e-7
    for u, l, L, Q, K, s in ((u1, x1, L1, Q1, 12, st[0]), (u2, x2, L2, Q2, 10, st[1])):
        for t, p, q, w in ((grad_op(u)[0], s["ph"], s["qh"], w_h), (grad_op(u)[1], s["pv"], s["qv"], w_v)):
            a, sg = np.abs(t), np.sign(t)
            assert np.all(np.where(a > tol, np.abs(p - w * sg), np.maximum(np.abs(p) - w, 0)) <= 1e-6)
            assert np.all(np.where(a < 2.0 - tol, np.abs(q), np.where(a > 2.0 + tol, np.abs(q - w * sg), 0)) <= 1e-6)
        g = -grad_op_T(s["ph"] - s["qh"], s["pv"] - s["qv"], u.shape)
        grad = L + Q * (u - l)
        lo, hi = np.maximum(l - 1.0, 0.0), np.minimum(l + 1.0, K - 1.0)
        resid = np.where(u >= hi - tol, np.maximum(grad - g, 0), np.where(u <= lo + tol, np.maximum(g - grad, 0),
                                                                           np.abs(g - grad)))
        assert resid.max() <= 1e-6, resid.max()
        assert np.abs(grad_op(u)[0]).max() > 2.0


def test_flow_pipeline_recovers_a_synthetic_flow():
    """The whole oracle pipeline on a small synthetic pair: cost volume, decoupled costs, two
    Dual_MM solves, refinement; the recovered displacement (label - offset) is within half
    a pixel of the true flow on most pixels (this fixes the sign conventions end to end)."""
    W, H, R = 40, 30, 3
    pair = synth.flow_pair(W, H, R - 0.5, seed=5, segments=3, slope=0.01, noise_sigma=0.0)
    K = 2 * R + 1
    D = flow.flow_cost_volume(pair.first, pair.second, K, K, R, R)
    w_h, w_v = cost_volume.contrast_weights(pair.first, lambda_pw=0.05)
    r = flow.solve_flow(D, w_h, w_v, 3, 8, RefineParams(C=3.0, n_warps=2, n_iters=20))
    # the true flow lives on the second image's grid; compare where it is locally smooth
    err = np.hypot(r.u1 - R - pair.flow[..., 0], r.u2 - R - pair.flow[..., 1])[3:-3, 3:-3]
    err_d = np.hypot(r.layer1.labels - R - pair.flow[..., 0], r.layer2.labels - R - pair.flow[..., 1])[3:-3, 3:-3]
    assert np.median(err) < 0.5, np.median(err)
    assert np.mean(err < 1.0) > 0.7
    assert np.median(err) < np.median(err_d)   # the refinement improves on the integer labels
