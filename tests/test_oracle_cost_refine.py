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


# ---------------------------------------------------------------- NL-PDHG, step by step
#
# A 1 x 3 grid (two horizontal edges), K = 8 labels, labels x = (1, 1, 5), C = 2, eps = 1,
# delta = 0, h = 1, tau = sigma = 1/4, w = (1/2, 1).  The costs give the slopes of the two-slope
# model (Sec. 3.1) s_L = D(x) - D(x-1), s_R = D(x+1) - D(x):
#   pixel 0: (s_L, s_R) = (-1, 2)   pixel 1: (-1/2, 1/4)   pixel 2: (-1, 2)
# (Au)_e = u_i - u_j, A^T y = (y0, y1 - y0, -y1).  R_- has alpha = 0, beta = C + delta - eps*delta
# = 2, so its conjugate prox (eq. pprox, step tau) is a soft threshold by tau*2 = 1/2 clamped to
# [-w, w]; R_+ has alpha = 1, beta = 0: a clamp to [-w, w].  One iteration (eq. cont_iterates):
#   u+ = prox_{tau D~}(u - tau A^T (p - q)),  q+ = prox(q + tau A u),  p+ = prox(p + sigma A(2u+ - u)).
# Iteration 1 (p = q = 0, u = u0 = (1, 1, 5)):
#   u_hat = u; every pixel lies in its dead zone [u0 + tau s_L, u0 + tau s_R]  ->  u+ = (1, 1, 5)
#   Au = (0, -4): q_hat = (0, -1) -> q = (0, -1/2);  p_hat = (0, -1) -> p = (0, -1)
# Iteration 2:
#   p - q = (0, -1/2), A^T(p - q) = (0, -1/2, 1/2), u_hat = (1, 9/8, 39/8)
#   pixel 1: 9/8 > u0 + tau s_R = 17/16 -> 9/8 - 1/16 = 17/16;  pixel 2: 39/8 in [19/4, 11/2] -> 5
#   u+ = (1, 17/16, 5)
#   q_hat = q + tau A u (the iterate before the step, Au = (0, -4)) = (0, -3/2) -> q = (0, -1)
#   2u+ - u = (1, 9/8, 5), A(.) = (-1/8, -31/8), p_hat = (-1/32, -1 - 31/32) -> p = (-1/32, -1)
PDHG_THETA = np.full((1, 3, 8), 5.0)
PDHG_THETA[0, 0, :3] = (2.0, 1.0, 3.0)
PDHG_THETA[0, 1, :3] = (1.5, 1.0, 1.25)
PDHG_THETA[0, 2, 4:7] = (2.0, 1.0, 3.0)
PDHG_LABELS = np.array([[1, 1, 5]])
PDHG_WH = np.array([[0.5, 1.0]])
PDHG_WV = np.zeros((0, 3))
PDHG_WANT = dict(u=np.array([[1.0, 17 / 16, 5.0]]), qh=np.array([[0.0, -1.0]]), ph=np.array([[-1 / 32, -1.0]]))


def _pdhg_two_iterations(mod):
    P = mod.RefineParams(C=2.0, eps=1.0, delta=0.0, h=1.0, tau=0.25, sigma=0.25, n_warps=1, n_iters=2)
    u, st = mod.refine_continuous(PDHG_THETA, PDHG_WH, PDHG_WV, PDHG_LABELS, P, return_state=True)
    return dict(u=u, qh=st["qh"], ph=st["ph"])


def test_pdhg_two_iterations_by_hand():
    """Two iterations from the labels, with the R_- (q) branch active on the edge across the
    step: every value is dyadic, so FP64 reproduces the hand computation exactly."""
    sL, sR = refine.linearize(PDHG_THETA, PDHG_LABELS.astype(np.float64), 1.0)
    np.testing.assert_array_equal(sL, [[-1.0, -0.5, -1.0]])
    np.testing.assert_array_equal(sR, [[2.0, 0.25, 2.0]])
    got = _pdhg_two_iterations(refine)
    for k, want in PDHG_WANT.items():
        np.testing.assert_array_equal(got[k], want, err_msg=k)


PDHG_MUTATIONS = {
    "q step with the wrong sign": [("qh = prox_conj(qh + P.tau * gh", "qh = prox_conj(qh - P.tau * gh"),
                                   ("qv = prox_conj(qv + P.tau * gv", "qv = prox_conj(qv - P.tau * gv")],
    "q step at u+ instead of u": [("gh, gv = grad_op(u)\n", "gh, gv = grad_op(u_new)\n")],
    "p step at u+ instead of 2u+ - u": [("grad_op(2.0 * u_new - u)", "grad_op(u_new)")],
    "A^T applied to p + q": [("grad_op_T(ph - qh, pv - qv", "grad_op_T(ph + qh, pv + qv")],
    "R_- threshold without the step": [("qh = prox_conj(qh + P.tau * gh, w_h, 0.0, beta_minus, P.tau)",
                                        "qh = prox_conj(qh + P.tau * gh, w_h, 0.0, beta_minus, 1.0)")],
}


@pytest.mark.parametrize("name", list(PDHG_MUTATIONS))
def test_pdhg_pin_catches_mutation(name):
    from tests.mutation import mutated
    got = _pdhg_two_iterations(mutated(refine, *PDHG_MUTATIONS[name]))
    assert any(not np.array_equal(got[k], v) for k, v in PDHG_WANT.items()), f"mutation '{name}' passes the pin"


def _criticality_violation(theta, w_h, w_v, labels, u, st, C, h=1.0):
    """Largest violation of the first-order conditions of min D~(u) + R_+(Au) - R_-(Au) at a
    fixed point (u, p, q) of the iteration, with eps = 1, delta = 0 (so R_+ = w|t| and
    R_- = w max(0, |t| - C)):  p in dR_+(Au), q in dR_-(Au), -A^T(p - q) in dD~(u) + N_box(u)."""
    K = theta.shape[2]
    u0 = labels.astype(np.float64)
    sL, sR = refine.linearize(theta, u0, h)
    lo, hi = np.maximum(u0 - h, 0.0), np.minimum(u0 + h, K - 1.0)
    viol = 0.0
    tol = 1e-9
    for t, p, q, w in ((refine.grad_op(u)[0], st["ph"], st["qh"], w_h), (refine.grad_op(u)[1], st["pv"], st["qv"], w_v)):
        a = np.abs(t)
        sgn = np.sign(t)
        # p in w * d|t|
        viol = max(viol, float(np.max(np.where(a > tol, np.abs(p - w * sgn), np.maximum(np.abs(p) - w, 0.0)), initial=0)))
        # q in w * d max(0, |t| - C): 0 inside, w sign(t) outside, between on the boundary
        inside = a < C - tol
        outside = a > C + tol
        qv = np.where(inside, np.abs(q), np.where(outside, np.abs(q - w * sgn),
                                                   np.maximum(np.maximum(-q * sgn, q * sgn - w), 0.0)))
        viol = max(viol, float(np.max(qv, initial=0)))
    g = -refine.grad_op_T(st["ph"] - st["qh"], st["pv"] - st["qv"], u.shape)
    # subdifferential of the two-slope model plus the box's normal cone, as an interval [gl, gu]
    gl = np.where(u > u0 + tol, sR, sL)
    gu = np.where(u < u0 - tol, sL, sR)
    gu = np.where(u >= hi - tol, np.inf, gu)
    gl = np.where(u <= lo + tol, -np.inf, gl)
    viol = max(viol, float(np.max(np.maximum(np.maximum(gl - g, g - gu), 0.0))))
    return viol


def _step_instance(seed=0):
    """3 x 4 grid, K = 10: two flat halves 5 labels apart (edges across the step keep |Au| > C),
    convex piecewise-linear costs with small random slopes, weights U[0.2, 0.6]."""
    g = np.random.default_rng(seed)
    H, W, K = 3, 4, 10
    x = np.where(np.arange(W)[None, :] < 2, 2, 7) + g.integers(0, 2, (H, W))
    sl = g.uniform(0.02, 0.2, (H, W, 1))
    sr = g.uniform(0.02, 0.2, (H, W, 1))
    d = np.arange(K)[None, None, :] - x[:, :, None]
    theta = np.where(d < 0, -d * sl, d * sr)
    return theta, g.uniform(0.2, 0.6, (H, W - 1)), g.uniform(0.2, 0.6, (H - 1, W)), x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pdhg_fixed_point_is_critical(seed):
    """Non-convex case (C = 2): the iteration reaches a fixed point that satisfies the
    first-order conditions of the DC problem (Sec. 2.4); with the q step's sign flipped it
    does not."""
    from tests.mutation import mutated
    theta, w_h, w_v, x = _step_instance(seed)
    bad = mutated(refine, *PDHG_MUTATIONS["q step with the wrong sign"])
    for mod, ok in ((refine, True), (bad, False)):
        P = mod.RefineParams(C=2.0, tau=0.25, sigma=0.25, n_warps=1, n_iters=800)
        u, st = mod.refine_continuous(theta, w_h, w_v, x, P, return_state=True)
        P.n_iters += 1
        u1, st1 = mod.refine_continuous(theta, w_h, w_v, x, P, return_state=True)
        residual = max(float(np.abs(u1 - u).max()), *(float(np.abs(st1[k] - st[k]).max()) for k in st))
        v = _criticality_violation(theta, w_h, w_v, x, u, st, 2.0)
        if ok:
            assert residual <= 1e-12 and v <= 1e-9, (residual, v)
            assert np.abs(refine.grad_op(u)[0]).max() > 2.0  # the truncation is active somewhere
        else:
            assert residual > 1e-12 or v > 1e-3, "sign-flipped q step passes the criticality check"
