"""Chain primitives in float64: messages, min-marginals and minorants.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Notation (paper App. A.1).  A chain has nodes 0..n-1 with unary cost vectors
a_j in R^K and edges (j, j+1) with pairwise cost w_j * rho(x_j - x_{j+1}),
where rho(t) = min(|t|, T) is the truncated-linear penalty obtained by
sampling the regulariser r at the label positions (Sec. 2.1, regulariser and
its figure; Sec. 2.2 "Stereo").  Potts is the case T = 1.

Arrays are batched over independent chains: ``a`` has shape (C, n, K) and
``w`` has shape (C, n-1).  Every function works on all C chains at once; the
loops along a chain follow the paper's order.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rho",
    "pairwise_table",
    "message",
    "message_bruteforce",
    "left_right_messages",
    "min_marginals",
    "chain_energy",
    "iterative_minorant",
    "naive_minorant",
    "hierarchical_minorant",
    "hierarchical_split",
    "chain_argmin",
    "uniform_minorant",
]


def rho(t, T: int):
    """Truncated-linear penalty min(|t|, T) (regulariser sampled at labels, Sec. 2.1)."""
    return np.minimum(np.abs(t), T)


def pairwise_table(K: int, T: int) -> np.ndarray:
    """K x K table rho(a - b) for labels a, b in {0..K-1}."""
    k = np.arange(K)
    return rho(k[:, None] - k[None, :], T).astype(np.float64)


def message_bruteforce(v: np.ndarray, w: np.ndarray, T: int) -> np.ndarray:
    """Message of the min-sum recursion, taken literally (App. A.1, eq. msg-pass).

    phi(b) = min_a [ v(a) + w * rho(a - b) ],  v: (C, K), w: (C,) -> (C, K).
    O(K^2) per chain; used as the definition against which ``message`` is pinned.
    """
    v = np.asarray(v, dtype=np.float64)
    K = v.shape[-1]
    P = pairwise_table(K, T)                       # P[a, b]
    return np.min(v[:, :, None] + np.asarray(w, np.float64)[:, None, None] * P[None], axis=1)


def message(v: np.ndarray, w: np.ndarray, T: int) -> np.ndarray:
    """Message phi(b) = min_a [v(a) + w rho(a-b)] written with the truncation made explicit.

    For |a - b| >= T the pairwise cost is the constant w*T, so
        phi(b) = min( min_{|a-b| < T} v(a) + w|a-b| ,  min_a v(a) + w T ).
    This is the same definition as ``message_bruteforce`` (no distance
    transform, no reordering), evaluated over the 2T-1 labels that can beat
    the truncation.  Requires w >= 0.
    """
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)[:, None]
    C, K = v.shape
    out = v.min(axis=1, keepdims=True) + w * T
    out = np.broadcast_to(out, (C, K)).copy()
    for d in range(-(T - 1), T):
        if abs(d) >= K:
            continue
        shifted = np.full((C, K), np.inf)
        # candidate a = b + d
        if d >= 0:
            shifted[:, : K - d] = v[:, d:]
        else:
            shifted[:, -d:] = v[:, : K + d]
        out = np.minimum(out, shifted + w * abs(d))
    return out


def left_right_messages(a: np.ndarray, w: np.ndarray, T: int):
    """Left and right min-marginal messages of chains (App. A.1 definitions).

    L[:, j] = phi_{j-1,j}: min over x_0..x_{j-1} of the part of the chain left of j
    R[:, j] = phi_{j+1,j}: min over x_{j+1}..x_{n-1} of the part right of j
    computed by the recursion phi_{j,j+1} = Msg(phi_{j-1,j} + a_j) (eq. msg-pass).
    """
    a = np.asarray(a, dtype=np.float64)
    C, n, K = a.shape
    L = np.zeros((C, n, K))
    R = np.zeros((C, n, K))
    for j in range(1, n):
        L[:, j] = message(L[:, j - 1] + a[:, j - 1], w[:, j - 1], T)
    for j in range(n - 2, -1, -1):
        R[:, j] = message(R[:, j + 1] + a[:, j + 1], w[:, j], T)
    return L, R


def min_marginals(a: np.ndarray, w: np.ndarray, T: int, normalized: bool = True) -> np.ndarray:
    """Min-marginals m_j = a_j + phi_{j-1,j} + phi_{j+1,j} (App. A.1, eq. min-marg-expression).

    With ``normalized`` the per-node minimum is subtracted (as in the paper's
    worked example of App. A.3.1), so each node's minimum is 0.
    """
    L, R = left_right_messages(a, w, T)
    m = np.asarray(a, np.float64) + L + R
    if normalized:
        m = m - m.min(axis=2, keepdims=True)
    return m


def chain_energy(a: np.ndarray, w: np.ndarray, T: int, x: np.ndarray) -> np.ndarray:
    """Energy of labelings x (C, n) of chains a (C, n, K): sum of unaries and pairwise terms."""
    a = np.asarray(a, np.float64)
    C, n, K = a.shape
    e = np.take_along_axis(a, x[:, :, None], axis=2)[:, :, 0].sum(axis=1)
    if n > 1:
        e = e + (np.asarray(w, np.float64) * rho(x[:, 1:] - x[:, :-1], T)).sum(axis=1)
    return e


def iterative_minorant(a: np.ndarray, w: np.ndarray, T: int, gammas) -> np.ndarray:
    """Iterative minorant of chains a (App. A.3.2, Alg. Iterative Minorant).

    Starting from h = 0 and the remainder r = a - h, the algorithm makes
    ``len(gammas)`` directional passes, forward on the first, then alternating
    ("reverse the chain").  At every node it forms the min-marginal of the
    remainder dynamically (message recursion + min-marginal expression) and
    moves the fraction gamma_s of it into the minorant.  The min-marginal is
    taken normalized (minimum over labels subtracted), so the remainder keeps
    the chain optimum and h >= 0.  The last gamma must be 1 for the result to
    be maximal (App. A.3, Lemma on maximal minorants).

    Before the first forward pass the right messages of the unmodified chain
    are computed by one backward message pass; during a pass the message
    arriving from the not-yet-visited side stays valid, because those nodes
    have not been modified since it was computed.

    Returns h with the shape of a.
    """
    a = np.asarray(a, dtype=np.float64)
    C, n, K = a.shape
    r = a.copy()
    h = np.zeros_like(r)
    L = np.zeros((C, n, K))
    R = np.zeros((C, n, K))
    for j in range(n - 2, -1, -1):
        R[:, j] = message(R[:, j + 1] + r[:, j + 1], w[:, j], T)
    for s, g in enumerate(gammas):
        if s % 2 == 0:
            order = range(n)
        else:
            order = range(n - 1, -1, -1)
        for j in order:
            m = r[:, j] + L[:, j] + R[:, j]
            d = g * (m - m.min(axis=1, keepdims=True))
            r[:, j] -= d
            h[:, j] += d
            if s % 2 == 0 and j + 1 < n:
                L[:, j + 1] = message(L[:, j] + r[:, j], w[:, j], T)
            if s % 2 == 1 and j - 1 >= 0:
                R[:, j - 1] = message(R[:, j] + r[:, j], w[:, j - 1], T)
    return h


def naive_minorant(a: np.ndarray, w: np.ndarray, T: int) -> np.ndarray:
    """Naive minorant: normalized min-marginals divided by the chain length (Sec. 2.3, App. A.1).

    This is the parallel block update obtained by splitting the chain into n
    copies of cost f/n, each contributing its min-marginal at one node.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[1]
    return min_marginals(a, w, T, normalized=True) / float(n)


def hierarchical_split(s: int, e: int) -> int:
    """Split node of the segment s..e (e > s): the segment breaks at the edge (i, i+1),
    the left part holding half of the nodes, rounded down (App. A.3.3: a chain of 32 is
    split into two chains of 16)."""
    return s + (e - s + 1) // 2 - 1


def hierarchical_minorant(a: np.ndarray, w: np.ndarray, T: int) -> np.ndarray:
    """Hierarchical minorant of chains a (App. A.3.3, Alg. Handshake and its figure).

    The chain is cut at the edge (i, i+1) in its middle.  With the message into i from
    the left part and the message into i+1 from the right part, the Handshake over that
    edge gives the left part half of the min-marginal at i (passed to the right as the
    message phi_ij into i+1) and bounces back, as phi_ji into i, what cannot be
    passed.  From then on the two parts are separate chains whose boundary unaries
    include these messages, and each is cut again in its middle; in a part, the
    messages computed at the level above stay valid on the side whose boundary did not
    change, and only the other side's messages are recomputed up to the new cut.  The
    recursion ends with single nodes; node k's minorant is its unary plus the two
    Handshake messages it received, its minimum subtracted (so h >= 0, as for the other
    minorants here, and the remainder a - h keeps the chain optimum when the minorant
    is exact).

    Arrays: a (C, n, K), w (C, n-1); returns h with the shape of a.
    """
    a = np.asarray(a, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    C, n, K = a.shape
    L = np.zeros((C, n, K))  # L[:, k]: message into k from the left, within k's current part
    R = np.zeros((C, n, K))  # R[:, k]: message into k from the right

    def handshake(i):
        j = i + 1
        phi_ji = message(a[:, j] + R[:, j], w[:, i], T)  # from j to i
        m_i = L[:, i] + a[:, i] + phi_ji                  # min-marginal at i
        phi_ij = message(m_i / 2.0 - phi_ji, w[:, i], T)  # a half of it shared to the right
        phi_ji = message(-phi_ij, w[:, i], T)             # what cannot be shared comes back
        R[:, i] = phi_ji
        L[:, j] = phi_ij

    def process(s, e):
        # on entry L is valid on s..i and R on i+1..e, i the split of s..e
        i = hierarchical_split(s, e)
        handshake(i)
        if i > s:
            i2 = hierarchical_split(s, i)
            for k in range(i, i2 + 1, -1):
                R[:, k - 1] = message(R[:, k] + a[:, k], w[:, k - 1], T)
            process(s, i)
        if e > i + 1:
            j2 = hierarchical_split(i + 1, e)
            for k in range(i + 1, j2):
                L[:, k + 1] = message(L[:, k] + a[:, k], w[:, k], T)
            process(i + 1, e)

    if n >= 2:
        i = hierarchical_split(0, n - 1)
        for k in range(0, i):
            L[:, k + 1] = message(L[:, k] + a[:, k], w[:, k], T)
        for k in range(n - 1, i + 1, -1):
            R[:, k - 1] = message(R[:, k] + a[:, k], w[:, k - 1], T)
        process(0, n - 1)
    m = a + L + R
    return m - m.min(axis=2, keepdims=True)


def chain_argmin(a: np.ndarray, w: np.ndarray, T: int) -> np.ndarray:
    """An optimal labeling of each chain (dynamic programming, App. A.1): x_0 minimises
    a_0 + R_0, then each x_j minimises a_j + R_j + w_{j-1} rho(x_{j-1} - x_j) given x_{j-1};
    the lowest label wins ties.  Returns (C, n) int64."""
    a = np.asarray(a, np.float64)
    w = np.asarray(w, np.float64)
    C, n, K = a.shape
    _, R = left_right_messages(a, w, T)
    x = np.zeros((C, n), np.int64)
    k = np.arange(K)
    x[:, 0] = np.argmin(a[:, 0] + R[:, 0], axis=1)
    for j in range(1, n):
        pw = w[:, j - 1][:, None] * rho(k[None, :] - x[:, j - 1][:, None], T)
        x[:, j] = np.argmin(a[:, j] + R[:, j] + pw, axis=1)
    return x


def uniform_minorant(a: np.ndarray, w: np.ndarray, T: int, *, tol: float = 1e-9, max_steps: int | None = None):
    """Maximal uniform minorant of chains a (App. A.3.1, Alg. Maximal Uniform Minorant).

    Starting from h = 0, repeat: take the normalized min-marginals m of the remainder
    f - h; stop when they are all 0; otherwise let O mark the label-nodes with m = 0 (the
    support of the remainder's optimal labelings), find the largest eps with
    eps * <1 - O, x> <= (f - h)(x) - min(f - h) for every labeling x (Prop. max-epsilon),
    and add eps to every label-node outside O.

    The largest eps is the minimum over labelings x with <1 - O, x> > 0 of the ratio
    N(x) / D(x), N(x) = (f - h)(x) - min(f - h), D(x) = <1 - O, x> (a minimum-ratio path,
    as the text notes).  It is found by Dinkelbach's parametric iteration: for a trial
    ratio e, an optimal labeling x of the chain with unaries (a - h) - e (1 - O) gives
    min_x [N(x) - e D(x)]; if that minimum is (numerically) 0, e is the largest eps,
    otherwise D(x) > 0 and the next trial is N(x) / D(x), strictly smaller.  The first
    trial is the smallest positive min-marginal, an upper bound of the largest eps (the
    best labeling through that label-node has N equal to it and D >= 1).

    ``tol`` (relative to the cost range) decides m = 0, the numerically delicate part that
    the text points out.  ``max_steps`` stops after that many outer steps (1 gives the
    first step of the worked example).  Arrays: a (C, n, K), w (C, n-1); returns h.
    """
    a = np.asarray(a, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    C, n, K = a.shape
    h = np.zeros_like(a)
    scale = max(1.0, float(np.abs(a).max()) if a.size else 1.0)
    eps_tol = tol * scale
    steps = 0
    # every step adds at least one label-node to the support O, so n*K steps suffice
    limit = n * K if max_steps is None else max_steps
    while steps < limit:
        rem = a - h
        m = min_marginals(rem, w, T, normalized=True)
        O = m <= eps_tol
        active = ~O.all(axis=(1, 2))
        if not active.any():
            break
        D = (~O).astype(np.float64)
        fstar = min_marginals(rem, w, T, normalized=False)[:, 0, :].min(axis=1)
        e = np.where(active, np.where(O, np.inf, m).reshape(C, -1).min(axis=1), 0.0)
        todo = active.copy()
        rounds = 0
        while todo.any():
            rounds += 1
            if rounds > 10 * n * K:  # Dinkelbach's ratios strictly decrease over finitely many labelings
                raise RuntimeError("uniform minorant: the parametric ratio search does not converge")
            x = chain_argmin(rem - e[:, None, None] * D, w, T)
            val = chain_energy(rem - e[:, None, None] * D, w, T, x) - fstar
            Dx = np.take_along_axis(D, x[:, :, None], axis=2)[:, :, 0].sum(axis=1)
            Nx = chain_energy(rem, w, T, x) - fstar
            better = todo & (val < -eps_tol) & (Dx > 0)
            e = np.where(better, Nx / np.where(Dx > 0, Dx, 1.0), e)
            todo = better
        h += np.where(active, e, 0.0)[:, None, None] * D
        steps += 1
    else:
        if max_steps is None:
            raise RuntimeError("uniform minorant: the support did not grow to every label-node")
    return h
