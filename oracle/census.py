"""Census transform, Hamming cost volume and left-right consistency check (float64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's data term for stereo is the Census transform of each image over a
small patch, compared by the pixel-wise Hamming distance (Sec. 3.1 "Stereo
Reconstruction", citing Zabih and Woodfill); outliers can be removed afterwards by
a two-sided (left-right) consistency check, which doubles the time (Sec. 4.1, its
comparison with a TV regulariser, and the caption of Table tab:timing).  The paper fixes neither the patch,
the comparison, the normalisation nor the check's rule; the readings taken here:

    census(I)(x, y)  = the bits [I(q) < I(x, y)] over the window positions q of the
                       (2r+1) x (2r+1) patch around (x, y) except the centre, in
                       raster order (dy outer, dx inner), coordinates clamped to
                       the image; n = (2r+1)^2 - 1 bits, window 3, 5 or 7
    left view        theta[y][x][d] = min(tau, H(cL(x, y), cR(x - d, y)) / n)
                     if x - d >= 0, else tau
    right view       theta[y][x][d] = min(tau, H(cR(x, y), cL(x + d, y)) / n)
                     if x + d < W, else tau
    (H = number of differing bits; tau in (0, 1], 1 = no truncation)

    left-right check: a left pixel with disparity u_L is kept iff its match
    x' = x - round(u_L) (round half up) lies in the image and
    |u_L(x, y) - u_R(x', y)| <= max_diff; otherwise it gets `invalid`.  The
    difference and the comparison are taken in FP64 (exact for FP32 disparities of
    the same magnitude), i.e. the plain definition.

The right view's edge weights are the contrast weights of the right image.
"""
from __future__ import annotations

import numpy as np

__all__ = ["census_bits", "census_codes", "census_cost_volume", "lr_check"]


def census_bits(I, window: int) -> np.ndarray:
    """[H][W][n] booleans: bit b of pixel (x, y) compares the b-th non-centre window
    position (raster order, clamped) with the centre: I(q) < I(x, y)."""
    I = np.asarray(I, np.float64)
    H, W = I.shape
    r = window // 2
    ys = np.arange(H)
    xs = np.arange(W)
    bits = []
    for dy in range(-r, r + 1):
        yy = np.clip(ys + dy, 0, H - 1)
        for dx in range(-r, r + 1):
            if dy == 0 and dx == 0:
                continue
            xx = np.clip(xs + dx, 0, W - 1)
            bits.append(I[yy][:, xx] < I)
    return np.stack(bits, axis=-1)


def census_codes(I, window: int) -> np.ndarray:
    """The census bits packed into one integer per pixel, bit b = census_bits[..., b]."""
    b = census_bits(I, window)
    codes = np.zeros(b.shape[:2], np.uint64)
    for k in range(b.shape[2]):
        codes |= b[:, :, k].astype(np.uint64) << np.uint64(k)
    return codes


def census_cost_volume(I_left, I_right, K: int, window: int = 5, trunc: float = 1.0,
                       view: str = "left") -> np.ndarray:
    """[H][W][K] Hamming cost volume of the left (or right) view, see the module text."""
    bl = census_bits(I_left, window)
    br = census_bits(I_right, window)
    H, W, n = bl.shape
    theta = np.full((H, W, K), float(trunc))
    for d in range(K):
        if view == "left":
            if d >= W:
                continue
            ham = np.count_nonzero(bl[:, d:, :] != br[:, :W - d, :], axis=-1)
            theta[:, d:, d] = np.minimum(trunc, ham / float(n))
        else:
            if d >= W:
                continue
            ham = np.count_nonzero(br[:, :W - d, :] != bl[:, d:, :], axis=-1)
            theta[:, :W - d, d] = np.minimum(trunc, ham / float(n))
    return theta


def lr_check(u_left, u_right, max_diff: float = 1.0, invalid: float = -1.0) -> np.ndarray:
    """Left disparities kept where the right view agrees (see the module text)."""
    uL = np.asarray(u_left, np.float64)
    uR = np.asarray(u_right, np.float64)
    H, W = uL.shape
    md = float(max_diff)
    out = np.full((H, W), float(invalid))
    for y in range(H):
        for x in range(W):
            xr = x - int(np.floor(uL[y, x] + 0.5))  # round half up
            if 0 <= xr < W and abs(uL[y, x] - uR[y, xr]) <= md:
                out[y, x] = uL[y, x]
    return out
