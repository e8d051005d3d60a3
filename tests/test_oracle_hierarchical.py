"""Pins of the oracle's hierarchical minorant (App. A.3.3, Alg. Handshake). No GPU."""
import itertools

import numpy as np
import pytest

import synth
from oracle import chain, dmm, energy


def _enumerate_chain(a, w, T):
    n, K = a.shape
    xs = np.array(list(itertools.product(range(K), repeat=n)), dtype=np.int64)
    e = a[np.arange(n)[None, :], xs].sum(axis=1)
    if n > 1:
        e = e + (w[None, :] * np.minimum(np.abs(xs[:, 1:] - xs[:, :-1]), T)).sum(axis=1)
    return xs, e


@pytest.mark.parametrize("n,K,T", [(1, 3, 2), (2, 3, 1), (3, 4, 2), (4, 3, 3), (5, 3, 1), (6, 3, 2), (7, 2, 1),
                                   (8, 3, 2)])
def test_minorant_inequality_and_exactness(n, K, T):
    """By enumeration: sum_k h_k(x_k) <= f(x) - f* for every labeling (a lower bound that
    keeps the optimum in the remainder), h >= 0, and h vanishes on an optimal labeling."""
    rng = np.random.default_rng(100 * n + 10 * K + T)
    C = 6
    a = rng.random((C, n, K))
    w = rng.random((C, max(n - 1, 0))) * 0.9
    h = chain.hierarchical_minorant(a, w, T)
    assert np.all(h >= 0.0) and np.allclose(h.min(axis=2), 0.0)
    for c in range(C):
        xs, e = _enumerate_chain(a[c], w[c], T)
        hs = h[c][np.arange(n)[None, :], xs].sum(axis=1)
        fstar = e.min()
        assert np.all(hs <= e - fstar + 1e-12)
        assert np.all(hs[e == fstar] <= 1e-12)


def test_zero_interaction_gives_the_unaries():
    rng = np.random.default_rng(4)
    a = rng.random((3, 9, 5))
    h = chain.hierarchical_minorant(a, np.zeros((3, 8)), 2)
    np.testing.assert_allclose(h, a - a.min(axis=2, keepdims=True), atol=1e-15)


def _msg(v, w, T):
    """min over a of v(a) + w min(|a - b|, T), by the definition."""
    K = v.shape[0]
    P = np.minimum(np.abs(np.arange(K)[:, None] - np.arange(K)[None, :]), T)
    return (v[:, None] + w * P).min(axis=0)


@pytest.mark.parametrize("seed", range(6))
def test_two_node_procedure_of_the_text(seed):
    """The two-node steps spelled out in App. A.3.3: lambda_1 = m_1 / 2, then the whole
    remaining min-marginal at node 2, then what remains at node 1 added to lambda_1."""
    rng = np.random.default_rng(seed)
    K, T = 4, 1 + seed % 3
    f1, f2, w = rng.random(K), rng.random(K), rng.random() * 0.7
    m1 = f1 + _msg(f2, w, T)
    lam1 = m1 / 2
    lam2 = _msg(f1 - lam1, w, T) + f2
    lam1 = lam1 + (f1 - lam1) + _msg(f2 - lam2, w, T)
    h = chain.hierarchical_minorant(np.stack([f1, f2])[None], np.array([[w]]), T)[0]
    np.testing.assert_allclose(h[0], lam1 - lam1.min(), atol=1e-14)
    np.testing.assert_allclose(h[1], lam2 - lam2.min(), atol=1e-14)


def test_split_pattern_of_the_figure():
    """A chain of 32 splits into halves down to 16 pieces of two (the figure of App. A.3.3)."""
    levels = [[(0, 31)]]
    while True:
        nxt = []
        for s, e in levels[-1]:
            if e > s + 1:
                i = chain.hierarchical_split(s, e)
                nxt += [(s, i), (i + 1, e)]
        if not nxt:
            break
        levels.append(nxt)
    assert [len(lv) for lv in levels] == [1, 2, 4, 8, 16]
    assert levels[-1] == [(2 * k, 2 * k + 1) for k in range(16)]
    assert levels[1] == [(0, 15), (16, 31)]


def test_per_node_constants_do_not_change_the_minorant():
    rng = np.random.default_rng(8)
    a = rng.random((2, 11, 6))
    w = rng.random((2, 10)) * 0.5
    c = rng.normal(size=(2, 11, 1)) * 3.0
    np.testing.assert_allclose(chain.hierarchical_minorant(a + c, w, 3), chain.hierarchical_minorant(a, w, 3),
                               atol=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_dual_mm_with_hierarchical_minorant_bruteforce(seed):
    """Dual_MM with the hierarchical minorant on 3x3, K = 3: LB <= min E after every
    half-step and never decreases (the minorant is exact, Sec. 2.3)."""
    T = 1 + seed % 2
    theta, w_h, w_v = synth.tiny_instance(3, 3, 3, seed=seed)
    emin, _ = energy.brute_force_min(theta, w_h, w_v, T)
    res = dmm.solve_discrete(theta, w_h, w_v, T, n_iters=4, minorant="hierarchical")
    assert np.all(res.lb_trace <= emin + 1e-9)
    assert np.all(np.diff(res.lb_trace) >= -1e-9)
    assert res.energy >= emin - 1e-9


def test_dual_mm_hierarchical_larger_grid_monotone():
    theta, w_h, w_v = synth.tiny_instance(6, 9, 4, seed=5, w_max=0.8)
    res = dmm.solve_discrete(theta, w_h, w_v, 2, n_iters=5, minorant="hierarchical")
    assert np.all(np.diff(res.lb_trace) >= -1e-9)
    assert res.lower_bound <= res.energy + 1e-9


def _from_scratch(a, w, T):
    """The same recursion with every part's messages recomputed from its two boundary
    messages (nothing reused from the level above), one chain (n, K)."""
    n, K = a.shape
    h = np.zeros_like(a)

    def part(s, e, lin, rin):
        if s == e:
            m = a[s] + lin + rin
            h[s] = m - m.min()
            return
        i = chain.hierarchical_split(s, e)
        Lm = lin
        for k in range(s, i):
            Lm = _msg(Lm + a[k], w[k], T)
        Rm = rin
        for k in range(e, i + 1, -1):
            Rm = _msg(Rm + a[k], w[k - 1], T)
        phi_ji = _msg(a[i + 1] + Rm, w[i], T)
        m_i = Lm + a[i] + phi_ji
        phi_ij = _msg(m_i / 2 - phi_ji, w[i], T)
        phi_ji = _msg(-phi_ij, w[i], T)
        part(s, i, lin, phi_ji)
        part(i + 1, e, phi_ij, rin)

    part(0, n - 1, np.zeros(K), np.zeros(K))
    return h


@pytest.mark.parametrize("n", [2, 3, 5, 9, 16, 23])
def test_reused_messages_equal_recomputed_ones(n):
    rng = np.random.default_rng(n)
    K, T = 5, 2
    a = rng.random((2, n, K))
    w = rng.random((2, n - 1)) * 0.6
    h = chain.hierarchical_minorant(a, w, T)
    for c in range(2):
        np.testing.assert_allclose(h[c], _from_scratch(a[c], w[c], T), atol=1e-12)
