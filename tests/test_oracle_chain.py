"""Pins of the oracle's chain primitives against the paper and against enumeration.

No GPU.  Each check is independent of the oracle's own arithmetic: printed
values of the paper, exhaustive enumeration of all labelings, or a closed form.
"""
import itertools

import numpy as np
import pytest

from oracle import chain


def _enumerate_chain(a, w, T):
    """All labelings of one chain a (n, K) with weights w (n-1,) and their energies."""
    n, K = a.shape
    xs = np.array(list(itertools.product(range(K), repeat=n)), dtype=np.int64)
    e = a[np.arange(n)[None, :], xs].sum(axis=1)
    if n > 1:
        e = e + (w[None, :] * np.minimum(np.abs(xs[:, 1:] - xs[:, :-1]), T)).sum(axis=1)
    return xs, e


def test_worked_example_min_marginals_potts5(golden):
    """App. A.3.1 example: printed normalized min-marginals for Potts strength 5."""
    g = golden("worked_example_potts5.txt")
    a = g["unaries"].T[None]                 # (1, 6 nodes, 3 labels)
    w = np.full((1, 5), 5.0)
    mm = chain.min_marginals(a, w, T=1)
    np.testing.assert_array_equal(mm[0].T, g["minmarg_w5"])


def test_worked_example_brute_force_agrees(golden):
    """The printed table is also what enumeration gives (pins the fixture itself)."""
    g = golden("worked_example_potts5.txt")
    a = g["unaries"].T
    xs, e = _enumerate_chain(a, np.full(5, 5.0), 1)
    n, K = a.shape
    mm = np.array([[e[xs[:, j] == k].min() for k in range(K)] for j in range(n)])
    mm -= mm.min(axis=1, keepdims=True)
    np.testing.assert_array_equal(mm.T, g["minmarg_w5"])


@pytest.mark.parametrize("K,T", [(1, 1), (2, 1), (5, 1), (5, 2), (7, 3), (6, 10), (12, 4)])
def test_message_window_equals_definition(K, T):
    g = np.random.default_rng(K * 31 + T)
    v = g.normal(size=(20, K)) * 3
    w = g.random(20) * 2
    np.testing.assert_allclose(chain.message(v, w, T), chain.message_bruteforce(v, w, T), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,K,T", [(1, 3, 1), (2, 3, 2), (4, 3, 1), (5, 4, 2), (6, 3, 3), (3, 5, 4)])
def test_min_marginals_match_enumeration(n, K, T):
    g = np.random.default_rng(100 * n + 10 * K + T)
    for _ in range(5):
        a = g.random((n, K)) * 4 - 1
        w = g.random(max(n - 1, 0)) * 2
        xs, e = _enumerate_chain(a, w, T)
        ref = np.array([[e[xs[:, j] == k].min() for k in range(K)] for j in range(n)])
        got = chain.min_marginals(a[None], w[None], T, normalized=False)[0]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
        # every node's min-marginal minimum is the chain optimum
        np.testing.assert_allclose(got.min(axis=1), e.min(), rtol=0, atol=1e-12)


GAMMAS = [(0.25, 0.25, 1.0), (1.0,), (0.5, 1.0), (0.25, 0.25, 0.25, 0.25, 0.25, 1.0)]


@pytest.mark.parametrize("gammas", GAMMAS)
@pytest.mark.parametrize("n,K,T", [(1, 3, 1), (2, 3, 1), (4, 3, 2), (5, 4, 1), (6, 3, 3)])
def test_iterative_minorant_properties(gammas, n, K, T):
    """Minorant (App. A.3 def.), exact at the optimum, maximal when the last gamma is 1."""
    g = np.random.default_rng(7 * n + 3 * K + T + len(gammas))
    for _ in range(4):
        a = g.random((n, K)) * 3
        w = g.random(max(n - 1, 0)) * 1.5
        h = chain.iterative_minorant(a[None], w[None], T, gammas)[0]
        xs, e = _enumerate_chain(a, w, T)
        hx = h[np.arange(n)[None, :], xs].sum(axis=1)
        assert np.all(h >= -1e-12)
        # modular minorant of f - min f: sum_j h_j(x_j) <= f(x) - f*
        assert np.all(hx <= e - e.min() + 1e-9)
        # exact at an optimum: h(x*) = 0
        assert hx[np.argmin(e)] == pytest.approx(0.0, abs=1e-9)
        # maximal: every normalized min-marginal of the remainder is zero (Lemma, App. A.3)
        rem = chain.min_marginals((a - h)[None], w[None], T, normalized=True)[0]
        np.testing.assert_allclose(rem, 0.0, atol=1e-9)


def test_iterative_minorant_zero_interaction_limit():
    """w = 0: chains decouple and the maximal minorant is a - min a (App. A.3.1, the w -> 0 limit)."""
    g = np.random.default_rng(5)
    a = g.random((3, 7, 5))
    w = np.zeros((3, 6))
    h = chain.iterative_minorant(a, w, 2, (0.25, 0.25, 1.0))
    np.testing.assert_allclose(h, a - a.min(axis=2, keepdims=True), atol=1e-12)


def test_iterative_minorant_partial_gamma_not_maximal():
    """With gamma < 1 on the last pass the remainder keeps slack (guards the gamma schedule)."""
    g = np.random.default_rng(9)
    a = g.random((1, 5, 4)) * 3
    w = np.full((1, 4), 0.2)
    h = chain.iterative_minorant(a, w, 2, (0.25,))
    rem = chain.min_marginals(a - h, w, 2, normalized=True)
    assert rem.max() > 1e-3


@pytest.mark.parametrize("n,K,T", [(3, 3, 1), (5, 4, 2)])
def test_naive_minorant_is_minorant(n, K, T):
    g = np.random.default_rng(n + K)
    a = g.random((n, K)) * 3
    w = g.random(n - 1)
    h = chain.naive_minorant(a[None], w[None], T)[0]
    xs, e = _enumerate_chain(a, w, T)
    hx = h[np.arange(n)[None, :], xs].sum(axis=1)
    assert np.all(hx <= e - e.min() + 1e-9)
    mm = np.array([[e[xs[:, j] == k].min() for k in range(K)] for j in range(n)])
    np.testing.assert_allclose(h, (mm - mm.min(axis=1, keepdims=True)) / n, atol=1e-12)
