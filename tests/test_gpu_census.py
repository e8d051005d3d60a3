"""GPU parity of the Census + Hamming cost volume and the left-right check against the
FP64 oracle, through the C ABI.

Cost volumes: bit-exact - every value is the correctly rounded quotient h / n (or the
truncation), so the GPU's FP32 value equals the oracle's FP64 value rounded to FP32,
and its FP16 value equals the oracle's value rounded to half.  Contrast weights of the
view's own image within 1e-6 relative.  Left-right check: bit-exact (its rounding is
exact, its comparison FP32 on both sides).
"""
import numpy as np
import pytest

import synth
from oracle import census as oc, cost_volume as ocv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1601_06274_amd as P
    return P


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _images(W, H, seed, levels):
    rng = np.random.default_rng(seed)
    IL, IR = rng.random((H, W)), rng.random((H, W))
    if levels:  # coarse intensities: many equal neighbours (a tie sets no bit)
        IL, IR = np.round(IL * levels) / levels, np.round(IR * levels) / levels
    return IL.astype(np.float32), IR.astype(np.float32)


def _expect(theta, dtype):
    return theta.astype(np.float16) if dtype == torch.float16 else theta.astype(np.float32)


CASES = [  # W, H, K, window, view, dtype, trunc, levels
    (37, 9, 13, 5, "left", torch.float32, 1.0, 0),
    (50, 7, 64, 3, "right", torch.float16, 1.0, 6),
    (33, 11, 100, 7, "left", torch.float16, 0.6, 4),
    (16, 4, 1, 5, "right", torch.float32, 1.0, 0),
    (20, 5, 256, 7, "right", torch.float32, 1.0, 3),   # K at its maximum, above W
    (1, 1, 3, 3, "left", torch.float32, 1.0, 0),       # one pixel
    (130, 6, 70, 5, "left", torch.float32, 0.5, 0),
    (97, 13, 65, 7, "right", torch.float16, 0.8, 0),
]


@pytest.mark.parametrize("W,H,K,window,view,dtype,trunc,levels", CASES)
def test_census_cost_volume_bitexact(W, H, K, window, view, dtype, trunc, levels):
    P = _need_gpu()
    print(f"[case] census W={W} H={H} K={K} window={window} view={view} {dtype} trunc={trunc}", flush=True)
    IL, IR = _images(W, H, 100 + W + K, levels)
    cost, w_h, w_v = P.build_cost_volume_census(_dev(IL), _dev(IR), K, window=window, trunc=trunc, view=view,
                                                dtype=dtype, lambda_pw=0.2, contrast_sigma=0.15)
    torch.cuda.synchronize()
    ref = oc.census_cost_volume(IL.astype(np.float64), IR.astype(np.float64), K, window=window,
                                trunc=float(np.float32(trunc)), view=view)
    np.testing.assert_array_equal(cost.cpu().numpy(), _expect(ref, dtype))
    own = IL if view == "left" else IR
    rw_h, rw_v = ocv.contrast_weights(own.astype(np.float64), lambda_pw=0.2, sigma_c=0.15)
    if W > 1:
        np.testing.assert_allclose(w_h.cpu().numpy(), rw_h, rtol=1e-6, atol=0)
    if H > 1:
        np.testing.assert_allclose(w_v.cpu().numpy(), rw_v, rtol=1e-6, atol=0)


def test_census_full_frame_sampled_rows():
    """1242 x 375, K = 192, FP16, 5 x 5 window, both views: rows at the top border, in the
    middle and at the bottom border against the oracle on bands of the frame (a band's
    inner rows see the same clamped windows as in the whole frame)."""
    P = _need_gpu()
    W, H, K, r = 1242, 375, 192, 2
    pair = synth.stereo_pair(W, H, K, seed=3000, segments=16, slope=0.08, occlusion_bands=4)
    IL, IR = pair.left.astype(np.float32), pair.right.astype(np.float32)
    for view in ("left", "right"):
        print(f"[case] census full frame view={view}", flush=True)
        cost, _, _ = P.build_cost_volume_census(_dev(IL), _dev(IR), K, window=2 * r + 1, view=view,
                                                dtype=torch.float16)
        torch.cuda.synchronize()
        got = cost.cpu().numpy()
        for y0, y1 in ((0, 6), (180, 186), (369, 375)):
            b0, b1 = max(0, y0 - r), min(H, y1 + r)
            ref = oc.census_cost_volume(IL[b0:b1].astype(np.float64), IR[b0:b1].astype(np.float64), K,
                                        window=2 * r + 1, view=view)
            np.testing.assert_array_equal(got[y0:y1], ref[y0 - b0:y1 - b0].astype(np.float16))


def _lr_compare(got, uL, uR, max_diff, invalid):
    """GPU check vs the FP64 oracle.  The kernel takes the difference and the comparison in
    FP32, so a pixel may differ only inside the tie band: its exact |u_L - u_R(x')| lies
    within one FP32 ulp of max_diff (where the rounded difference can fall on either side of
    the bound).  Every other pixel is equal.  Returns the number of tie-band differences."""
    ref = oc.lr_check(uL, uR, max_diff=max_diff, invalid=invalid)
    diff = got != ref
    if not diff.any():
        return 0
    H, W = uL.shape
    ys, xs = np.nonzero(diff)
    xr = xs - np.floor(uL[ys, xs].astype(np.float64) + 0.5).astype(np.int64)
    assert np.all((xr >= 0) & (xr < W)), "a differing pixel matches outside the image"
    exact = np.abs(uL[ys, xs].astype(np.float64) - uR[ys, xr].astype(np.float64))
    ulp = float(np.spacing(np.float32(max_diff))) if max_diff > 0 else float(np.finfo(np.float32).tiny)
    band = np.abs(exact - max_diff) <= ulp
    assert band.all(), f"{int((~band).sum())} pixels differ outside the FP32 tie band"
    # within the band the GPU keeps the pixel exactly when its FP32 difference passes
    d32 = np.abs(uL[ys, xs] - uR[ys, xr]).astype(np.float32)
    keep32 = d32 <= np.float32(max_diff)
    np.testing.assert_array_equal(got[ys, xs], np.where(keep32, uL[ys, xs], np.float32(invalid)))
    return int(diff.sum())


def test_lr_check_against_fp64():
    P = _need_gpu()
    rng = np.random.default_rng(77)
    H, W = 23, 301
    uL = (rng.random((H, W)) * 40).astype(np.float32)
    uL[:, ::7] = np.round(uL[:, ::7]) + 0.5           # half-integers: round half up
    uL[:, ::11] = np.round(uL[:, ::11])
    uL[0, :5] = np.array([0.0, 0.49999997, 0.5, 1e9, -3.0], np.float32)  # far outside, negative
    uR = (uL + rng.normal(0, 1.0, (H, W))).astype(np.float32)   # same grid, roughly consistent
    uR[:, 50:80] = rng.random((H, 30)).astype(np.float32) * 40   # an inconsistent band
    uR[3, :] = uL[3, :] + np.float32(1.0)                        # differences at the bound (rounded)
    # exact differences within one FP32 ulp of the bound 1, where FP32 rounding decides:
    # u_L in [0.5, 1) matches x - 1, and u_R there is u_L + 1 rounded to FP32
    uL[4] = (0.5 + rng.random(W) * 0.5).astype(np.float32)
    uR[4, :-1] = (uL[4, 1:] + np.float32(1.0)).astype(np.float32)
    for md in (1.0, 0.0, 2.5):
        print(f"[case] lr_check H={H} W={W} max_diff={md}", flush=True)
        out = P.lr_check(_dev(uL), _dev(uR), max_diff=md, invalid=-7.0)
        torch.cuda.synchronize()
        n_tie = _lr_compare(out.cpu().numpy(), uL, uR, md, -7.0)
        print(f"[parity] lr_check max_diff={md}: {n_tie} tie-band pixels decided by FP32 rounding", flush=True)


def test_left_right_pipeline():
    """Census volumes of both views, Dual_MM labels of both, then the check: the GPU's
    check of the GPU's labels equals the oracle's check of the same labels, most pixels
    of a textured synthetic pair pass, and the occluded left border is rejected."""
    P = _need_gpu()
    W, H, K = 320, 96, 48
    pair = synth.stereo_pair(W, H, K, seed=2100, segments=6, slope=0.02, occlusion_bands=0)
    IL, IR = _dev(pair.left.astype(np.float32)), _dev(pair.right.astype(np.float32))
    labs = {}
    for view in ("left", "right"):
        print(f"[case] pipeline view={view}", flush=True)
        cost, w_h, w_v = P.build_cost_volume_census(IL, IR, K, window=5, view=view, dtype=torch.float16,
                                                    lambda_pw=0.05)
        res = P.solve_discrete(cost, w_h, w_v, T=3, n_iters=10)
        labs[view] = res.labels.float()
    out = P.lr_check(labs["left"], labs["right"], max_diff=1.0, invalid=-1.0)
    torch.cuda.synchronize()
    uL, uR, got = labs["left"].cpu().numpy(), labs["right"].cpu().numpy(), out.cpu().numpy()
    n_tie = _lr_compare(got, uL, uR, 1.0, -1.0)
    print(f"[parity] left-right pipeline: {n_tie} tie-band pixels", flush=True)
    kept = got >= 0
    assert kept.mean() > 0.5, kept.mean()
    x = np.arange(W)[None, :]
    assert not np.any(kept & (x - uL < -0.5))  # a match left of the image is never kept
