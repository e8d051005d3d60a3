"""Pins of the oracle's Dual_MM against weak duality, enumeration and chain exactness. No GPU."""
import numpy as np
import pytest

import synth
from oracle import chain, dmm, energy


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_3x3_weak_duality_and_monotone(seed):
    """LB <= min E <= E(x_out) after every half-step (Sec. 2.3 weak duality); LB never decreases."""
    T = 1 + seed % 2
    theta, w_h, w_v = synth.tiny_instance(3, 3, 3, seed=seed)
    emin, _ = energy.brute_force_min(theta, w_h, w_v, T)
    res = dmm.solve_discrete(theta, w_h, w_v, T, n_iters=4)
    lb0 = dmm.lower_bound(theta, np.zeros_like(theta, dtype=np.float64), w_h, w_v, T)
    trace = np.concatenate([[lb0], res.lb_trace])
    assert np.all(trace <= emin + 1e-9)
    assert np.all(np.diff(trace) >= -1e-9)
    assert res.energy >= emin - 1e-9
    assert res.energy == pytest.approx(energy.grid_energy(theta, w_h, w_v, T, res.labels))
    assert res.lower_bound == pytest.approx(res.lb_trace[-1])


@pytest.mark.parametrize("minorant", ["iterative", "naive"])
def test_lb_monotone_larger_grid(minorant):
    theta, w_h, w_v = synth.tiny_instance(6, 7, 4, seed=3, w_max=0.8)
    res = dmm.solve_discrete(theta, w_h, w_v, 2, n_iters=5, minorant=minorant)
    assert np.all(np.diff(res.lb_trace) >= -1e-9)
    assert res.lower_bound <= res.energy + 1e-9


def test_single_column_reaches_optimum_after_one_iteration():
    """W = 1: F is modular, G one chain; the chain LP is tight (App. A.2), so LB = min E at once."""
    for seed in range(5):
        theta, w_h, w_v = synth.tiny_instance(6, 1, 3, seed=seed)
        emin, _ = energy.brute_force_min(theta, w_h, w_v, 2)
        res = dmm.solve_discrete(theta, w_h, w_v, 2, n_iters=1)
        assert res.lb_trace[0] == pytest.approx(emin, abs=1e-12)
        assert res.lower_bound == pytest.approx(emin, abs=1e-12)


def test_single_row_labels_are_optimal():
    """H = 1: the output labeling is an exact chain optimum (unique optimum with random costs)."""
    theta, w_h, w_v = synth.tiny_instance(1, 7, 3, seed=11)
    emin, xbest = energy.brute_force_min(theta, w_h, w_v, 1)
    res = dmm.solve_discrete(theta, w_h, w_v, 1, n_iters=2)
    assert res.energy == pytest.approx(emin, abs=1e-12)
    np.testing.assert_array_equal(res.labels, xbest)


def test_h_half_step_leaves_rows_maximal():
    """After a horizontal half-step (last gamma = 1) all normalized row min-marginals of F are 0."""
    theta, w_h, w_v = synth.tiny_instance(4, 6, 5, seed=2)
    lam = dmm.half_step(theta, np.zeros(theta.shape), w_h, w_v, 2, "h")
    mm = chain.min_marginals(theta - lam, w_h, 2, normalized=True)
    np.testing.assert_allclose(mm, 0.0, atol=1e-9)
    # and the move went to G: lambda >= 0 (minorant of F is non-negative)
    assert lam.min() >= -1e-12


def test_decomposition_identity():
    """F(x) + G(x) = E(x) for every lambda: check on random labelings."""
    theta, w_h, w_v = synth.tiny_instance(4, 5, 3, seed=8)
    res = dmm.solve_discrete(theta, w_h, w_v, 2, n_iters=2)
    g = np.random.default_rng(0)
    for _ in range(10):
        x = g.integers(0, 3, size=(4, 5))
        F = chain.chain_energy(theta - res.lam, w_h, 2, x).sum()
        G = chain.chain_energy(np.transpose(res.lam, (1, 0, 2)), w_v.T, 2, x.T).sum()
        assert F + G == pytest.approx(energy.grid_energy(theta, w_h, w_v, 2, x), abs=1e-9)


def test_warm_start_resume_equals_continuous_run():
    """5 iterations, then 5 more from the saved lambda, equals 10 iterations."""
    theta, w_h, w_v = synth.tiny_instance(5, 5, 4, seed=4)
    a = dmm.solve_discrete(theta, w_h, w_v, 2, n_iters=5)
    b = dmm.solve_discrete(theta, w_h, w_v, 2, n_iters=5, lam0=a.lam)
    c = dmm.solve_discrete(theta, w_h, w_v, 2, n_iters=10)
    np.testing.assert_allclose(b.lam, c.lam, atol=1e-12)
    np.testing.assert_array_equal(b.labels, c.labels)


def test_lb_below_lp_relaxation():
    """The dual bound never exceeds the LP relaxation optimum (the dual's maximum, Sec. 2.3)."""
    from scipy.optimize import linprog
    theta, w_h, w_v = synth.tiny_instance(3, 3, 3, seed=21)
    T = 1
    H, W, K = theta.shape
    nodes = [(y, x) for y in range(H) for x in range(W)]
    edges = [((y, x), (y, x + 1), w_h[y, x]) for y in range(H) for x in range(W - 1)]
    edges += [((y, x), (y + 1, x), w_v[y, x]) for y in range(H - 1) for x in range(W)]
    nid = {p: i for i, p in enumerate(nodes)}
    nv = len(nodes) * K
    ne = len(edges) * K * K
    c = np.concatenate([theta.reshape(-1).astype(np.float64),
                        np.concatenate([wgt * chain.pairwise_table(K, T).reshape(-1) for _, _, wgt in edges])])
    A_eq, b_eq = [], []
    for i in range(len(nodes)):
        row = np.zeros(nv + ne); row[i * K:(i + 1) * K] = 1; A_eq.append(row); b_eq.append(1)
    for e, (p, q, _) in enumerate(edges):
        base = nv + e * K * K
        for a in range(K):
            row = np.zeros(nv + ne); row[base + a * K: base + (a + 1) * K] = 1; row[nid[p] * K + a] = -1
            A_eq.append(row); b_eq.append(0)
        for b in range(K):
            row = np.zeros(nv + ne); row[base + b: base + K * K: K] = 1; row[nid[q] * K + b] = -1
            A_eq.append(row); b_eq.append(0)
    lp = linprog(c, A_eq=np.array(A_eq), b_eq=np.array(b_eq), bounds=(0, None), method="highs")
    assert lp.status == 0
    res = dmm.solve_discrete(theta, w_h, w_v, T, n_iters=10)
    assert res.lb_trace.max() <= lp.fun + 1e-7
