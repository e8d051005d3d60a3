"""Pins of the oracle's Census / Hamming cost volume and left-right check. No GPU."""
import numpy as np
import pytest

from oracle import census


def _brute_cost(IL, IR, K, window, trunc, view):
    """Cost volume by direct pairwise comparison counts (no bit codes, no popcount)."""
    H, W = IL.shape
    r = window // 2
    n = window * window - 1
    out = np.full((H, W, K), float(trunc))

    def bit(I, y, x, dy, dx):
        yy = min(max(y + dy, 0), H - 1)
        xx = min(max(x + dx, 0), W - 1)
        return I[yy, xx] < I[y, x]

    for y in range(H):
        for x in range(W):
            for d in range(K):
                xo = x - d if view == "left" else x + d
                if not 0 <= xo < W:
                    continue
                A, B = (IL, IR) if view == "left" else (IR, IL)
                diff = 0
                for dy in range(-r, r + 1):
                    for dx in range(-r, r + 1):
                        if dy or dx:
                            diff += bit(A, y, x, dy, dx) != bit(B, y, xo, dy, dx)
                out[y, x, d] = min(trunc, diff / n)
    return out


def test_bright_dot_fixes_the_comparison_direction():
    # a single bright pixel: every neighbour is darker, so its code has all n bits;
    # its neighbours see one brighter and otherwise equal pixels: no bit
    I = np.zeros((9, 9))
    I[4, 4] = 1.0
    for w in (3, 5, 7):
        c = census.census_codes(I, w)
        n = w * w - 1
        assert int(c[4, 4]) == (1 << n) - 1
        assert int(c[4, 5]) == 0 and int(c[3, 4]) == 0
        assert int(c[0, 0]) == 0


def test_constant_images_cost_nothing():
    I = np.full((6, 10), 0.3)
    th = census.census_cost_volume(I, I, 4, window=5)
    assert np.all(th[:, 3:, :] == 0.0)
    # matches outside the image cost the truncation
    assert np.all(th[:, 0, 1:] == 1.0)


@pytest.mark.parametrize("window,view", [(3, "left"), (5, "left"), (5, "right"), (7, "right"), (7, "left")])
def test_cost_volume_against_pairwise_counts(window, view):
    rng = np.random.default_rng(11 + window)
    IL = np.round(rng.random((7, 12)) * 8) / 8  # coarse levels: many equal intensities
    IR = np.round(rng.random((7, 12)) * 8) / 8
    K, trunc = 5, 0.75
    th = census.census_cost_volume(IL, IR, K, window=window, trunc=trunc, view=view)
    np.testing.assert_array_equal(th, _brute_cost(IL, IR, K, window, trunc, view))


def test_rank_transform_is_invariant_to_monotone_intensity_maps():
    rng = np.random.default_rng(3)
    IL, IR = rng.random((8, 16)), rng.random((8, 16))
    f = lambda I: I ** 3 + 0.5 * I - 2.0  # strictly increasing
    a = census.census_cost_volume(IL, IR, 6, window=5)
    b = census.census_cost_volume(f(IL), f(IR), 6, window=5)
    np.testing.assert_array_equal(a, b)


def test_true_shift_costs_zero_away_from_the_borders():
    rng = np.random.default_rng(5)
    s, W, H, r = 4, 24, 9, 2
    J = rng.random((H, W + s))
    IL, IR = J[:, :W], J[:, s:s + W]  # I_R(x') = I_L(x' + s)
    th = census.census_cost_volume(IL, IR, 8, window=2 * r + 1)
    inner = th[:, s + r:W - r, s]
    assert np.all(inner == 0.0)
    assert np.all(th[:, s + r:W - r, s + 1] > 0.0)  # the neighbouring disparity does not match


def test_right_view_compares_the_same_pixel_pairs():
    rng = np.random.default_rng(9)
    IL, IR = rng.random((6, 15)), rng.random((6, 15))
    K = 7
    L = census.census_cost_volume(IL, IR, K, window=5, view="left")
    R = census.census_cost_volume(IL, IR, K, window=5, view="right")
    for d in range(K):
        np.testing.assert_array_equal(R[:, :15 - d, d], L[:, d:, d])
        assert np.all(R[:, 15 - d:, d] == 1.0)


def test_lr_check_cases():
    H, W = 3, 10
    uL = np.full((H, W), 3.0)
    uR = np.full((H, W), 3.0)
    out = census.lr_check(uL, uR, max_diff=1.0, invalid=-1.0)
    assert np.all(out[:, :3] == -1.0) and np.all(out[:, 3:] == 3.0)
    uR2 = uR.copy()
    uR2[1, 4] = 4.0   # |3 - 4| = 1: kept (bound inclusive)
    uR2[2, 4] = 4.5   # 1.5: rejected
    out = census.lr_check(uL, uR2, max_diff=1.0, invalid=-1.0)
    assert out[1, 7] == 3.0 and out[2, 7] == -1.0
    # the match column rounds half up: 2.5 -> 3
    uL3 = np.full((1, 6), 2.5)
    uR3 = np.array([[0.0, 0.0, 2.5, 9.0, 9.0, 9.0]])
    out = census.lr_check(uL3, uR3, max_diff=0.25, invalid=-1.0)
    assert out[0, 5] == 2.5 and out[0, 4] == -1.0 and out[0, 3] == -1.0
