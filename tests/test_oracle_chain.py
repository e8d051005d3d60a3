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


# ---------------------------------------------------------------- Alg. Iterative Minorant, step by step
#
# A 3-node chain with 2 labels, Potts (T = 1), w = 2 on both edges, unaries (label 0, label 1):
#   node 0: (1, 4)   node 1: (0, 2)   node 2: (0, 3)
# f(x) = sum_j a_j(x_j) + 2 [x0 != x1] + 2 [x1 != x2].  All eight labelings (x0 x1 x2):
#   000: 1  001: 6  010: 7  011: 8  100: 6  101: 11  110: 8  111: 9
# Alg. Iterative Minorant (App. A.3.2) with gamma = (1/4, 1): pass 1 visits nodes 0, 1, 2 (the
# chain in its given order), pass 2 the reversed chain 2, 1, 0.  At each node the min-marginal of
# the current remainder f - h is taken (normalized to minimum 0) and the fraction gamma_s of it
# is moved into h_j:
#   pass 1, node 0: m = (1, 6) -> (0, 5);   h0 += (0, 5/4)
#           node 1: remainder 100: 19/4, 101: 39/4, 110: 27/4, 111: 31/4, others as above;
#                   m = (1, 27/4) -> (0, 23/4); h1 += (0, 23/16)
#           node 2: remainder 010: 89/16, 110: 85/16, 011: 105/16, 111: 101/16;
#                   m = (1, 6) -> (0, 5);   h2 += (0, 5/4)
#   pass 2, node 2: remainder 001: 19/4, 101: 17/2, 011: 85/16, 111: 81/16;
#                   m = (1, 19/4) -> (0, 15/4); h2 += (0, 15/4)
#           node 1: remainder 011: 25/16, 111: 21/16, 001: 1;
#                   m = (1, 21/16) -> (0, 5/16); h1 += (0, 5/16)
#           node 0: m = (1, 1) -> (0, 0)
#   h = [(0, 5/4), (0, 7/4), (0, 5)]
# With gamma = (1/4, 1/4, 1) (a third pass in the original order) the same steps give
#   h = [(0, 115/32), (0, 71/32), (0, 35/16)].
# Visiting the reversed chain first would give the mirror images [(0, 5), (0, 7/4), (0, 5/4)] and
# [(0, 35/16), (0, 71/32), (0, 115/32)]: the pass order matters here, so these values pin it.
PIN_A = np.array([[1.0, 4.0], [0.0, 2.0], [0.0, 3.0]])
PIN_W = np.array([2.0, 2.0])
PIN_H = {
    (0.25, 1.0): np.array([[0, 5 / 4], [0, 7 / 4], [0, 5]]),
    (0.25, 0.25, 1.0): np.array([[0, 115 / 32], [0, 71 / 32], [0, 35 / 16]]),
}


def _iterative_by_enumeration(a, w, T, gammas, first_forward=True):
    """Alg. Iterative Minorant with every min-marginal taken from its definition (App. A.1:
    the minimum of the remainder over all labelings through (j, k)), by enumeration."""
    n, K = a.shape
    r = a.astype(np.float64).copy()
    h = np.zeros_like(r)
    for s, g in enumerate(gammas):
        forward = (s % 2 == 0) == first_forward
        for j in (range(n) if forward else range(n - 1, -1, -1)):
            xs, e = _enumerate_chain(r, w, T)
            m = np.array([e[xs[:, j] == k].min() for k in range(K)])
            d = g * (m - m.min())
            r[j] -= d
            h[j] += d
    return h


@pytest.mark.parametrize("gammas", list(PIN_H))
def test_iterative_minorant_hand_worked(gammas):
    """The oracle reproduces the hand-worked steps exactly (dyadic values, exact in FP64)."""
    h = chain.iterative_minorant(PIN_A[None], PIN_W[None], 1, gammas)[0]
    np.testing.assert_array_equal(h, PIN_H[gammas])
    # the enumeration form of the algorithm agrees, and visiting the reversed chain first
    # does not: the pin discriminates the pass order
    np.testing.assert_array_equal(_iterative_by_enumeration(PIN_A, PIN_W, 1, gammas), PIN_H[gammas])
    back = _iterative_by_enumeration(PIN_A, PIN_W, 1, gammas, first_forward=False)
    np.testing.assert_array_equal(back, PIN_H[gammas][::-1])
    assert not np.array_equal(back, PIN_H[gammas])


@pytest.mark.parametrize("n,K,T", [(2, 3, 1), (3, 3, 2), (4, 2, 1), (4, 3, 3), (5, 3, 2)])
@pytest.mark.parametrize("gammas", [(0.25, 1.0), (0.25, 0.25, 1.0), (0.5, 0.25, 0.75, 1.0)])
def test_iterative_minorant_equals_enumeration_form(n, K, T, gammas):
    """Message recursion (the oracle) vs min-marginals by enumeration, on random chains."""
    g = np.random.default_rng(11 * n + 5 * K + T + len(gammas))
    for _ in range(3):
        a = np.round(g.random((n, K)) * 8) / 2
        w = np.round(g.random(n - 1) * 6) / 4
        h = chain.iterative_minorant(a[None], w[None], T, gammas)[0]
        np.testing.assert_allclose(h, _iterative_by_enumeration(a, w, T, gammas), rtol=0, atol=1e-12)


ITERATIVE_MUTATIONS = {
    "reversed chain first": ("order = range(n)\n        else:\n            order = range(n - 1, -1, -1)",
                             "order = range(n - 1, -1, -1)\n        else:\n            order = range(n)"),
    "gamma schedule reversed": ("for s, g in enumerate(gammas):", "for s, g in enumerate(tuple(gammas)[::-1]):"),
    "message from the unmodified unary": ("L[:, j + 1] = message(L[:, j] + r[:, j]",
                                          "L[:, j + 1] = message(L[:, j] + a[:, j]"),
    "min-marginal not normalized": ("d = g * (m - m.min(axis=1, keepdims=True))", "d = g * m"),
}


@pytest.mark.parametrize("name", list(ITERATIVE_MUTATIONS))
def test_iterative_minorant_pin_catches_mutation(name):
    """Each planted mistake in a copy of the oracle fails the hand-worked pin."""
    from tests.mutation import mutated
    mut = mutated(chain, ITERATIVE_MUTATIONS[name])
    failed = 0
    for gammas, want in PIN_H.items():
        h = mut.iterative_minorant(PIN_A[None], PIN_W[None], 1, gammas)[0]
        failed += not np.array_equal(h, want)
    assert failed >= 1, f"mutation '{name}' passes the pin"
