"""SAD cost volume and contrast-weighted edge strengths (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper samples the data term D_i at every label to obtain the unary cost
vectors f_i (Sec. 2.2 "Stereo"; the cost volume is precomputed for all
labels, Sec. 1 and Table tab:timing "Cost Vol.").  The paper's own data term
is Census + Hamming (Sec. 3.1); the workloads here use a truncated 3x3 sum of
absolute differences instead, with the same role:

    e(x, y, d)       = |I_L(x, y) - I_R(x - d, y)|        if x - d >= 0
                     = tau                                 otherwise
    theta[y][x][d]   = min(tau, (1/|N|) sum_{(x',y') in N(x,y)} e(x', y', d))

with N(x, y) the window x-r..x+r, y-r..y+r clamped to the image (clamp to
edge), r = window // 2, tau the truncation.

Edge strengths w_ij are image dependent and lower across strong edges
(Sec. 2.1, below eq. regularizer-form):

    w_h[y][x] = lambda_pw * exp(-|I_L(x+1, y) - I_L(x, y)| / sigma_c)
    w_v[y][x] = lambda_pw * exp(-|I_L(x, y+1) - I_L(x, y)| / sigma_c)
"""
from __future__ import annotations

import numpy as np

__all__ = ["sad_cost_volume", "contrast_weights", "round_half"]


def sad_cost_volume(I_left, I_right, K: int, window: int = 3, trunc: float = 0.3) -> np.ndarray:
    L = np.asarray(I_left, np.float64)
    Rr = np.asarray(I_right, np.float64)
    H, W = L.shape
    r = window // 2
    theta = np.zeros((H, W, K))
    xs = np.arange(W)
    for d in range(K):
        e = np.full((H, W), trunc)
        valid = xs - d >= 0
        e[:, valid] = np.abs(L[:, valid] - Rr[:, xs[valid] - d])
        acc = np.zeros((H, W))
        for dy in range(-r, r + 1):
            yy = np.clip(np.arange(H) + dy, 0, H - 1)
            for dx in range(-r, r + 1):
                xx = np.clip(xs + dx, 0, W - 1)
                acc += e[yy][:, xx]
        theta[:, :, d] = np.minimum(trunc, acc / float(window * window))
    return theta


def contrast_weights(I_left, lambda_pw: float = 0.1, sigma_c: float = 0.1):
    L = np.asarray(I_left, np.float64)
    w_h = lambda_pw * np.exp(-np.abs(L[:, 1:] - L[:, :-1]) / sigma_c)
    w_v = lambda_pw * np.exp(-np.abs(L[1:, :] - L[:-1, :]) / sigma_c)
    return w_h, w_v


def round_half(x) -> np.ndarray:
    """Round to IEEE binary16 with round-to-nearest-even, returned as float64."""
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)
