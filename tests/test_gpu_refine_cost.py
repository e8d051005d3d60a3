"""GPU parity of dm_refine_continuous and dm_build_cost_volume against the FP64 oracle.

Refinement: both sides start from the same labels (the oracle's); |u_gpu - u_ref| <= 1e-4.
Cost volume: FP32 output within 2e-6 absolute of the FP64 definition; FP16 output equal
to the FP64 value rounded to half, up to one half-precision ulp (the GPU rounds its FP32
result); contrast weights within 1e-6 relative.
"""
import numpy as np
import pytest

import synth
from oracle import cost_volume as ocv, dmm as odmm, refine as oref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U_TOL = 1e-4


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1601_06274_amd as P
    return P


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _refine_case(theta, w_h, w_v, labels, P_ref, theta_dtype=torch.float32, name=""):
    P = _need_gpu()
    print(f"[case] {name} shape={theta.shape} warps={P_ref.n_warps} iters={P_ref.n_iters} C={P_ref.C} "
          f"eps={P_ref.eps} delta={P_ref.delta} {theta_dtype}", flush=True)
    th = _dev(theta, theta_dtype)
    th_used = th.float().cpu().numpy().astype(np.float64)
    u = P.refine_continuous(th, _dev(labels, torch.int32), _dev(w_h), _dev(w_v), C=P_ref.C, eps=P_ref.eps,
                            delta=P_ref.delta, h=P_ref.h, tau=P_ref.tau, sigma=P_ref.sigma, n_warps=P_ref.n_warps,
                            n_iters=P_ref.n_iters)
    torch.cuda.synchronize()
    # the C ABI takes float32 parameters: give the oracle the same (rounded) values
    P32 = oref.RefineParams(**{k: (float(np.float32(v)) if isinstance(v, float) else v)
                              for k, v in vars(P_ref).items()})
    u_ref = oref.refine_continuous(th_used, w_h.astype(np.float64), w_v.astype(np.float64), labels, P32)
    err = np.abs(u.cpu().numpy() - u_ref)
    print(f"[parity] {name}: u_err_max={err.max():.3e} u_err_mean={err.mean():.3e} "
          f"moved={float(np.abs(u_ref - labels).mean()):.3e}", flush=True)
    return err


@pytest.mark.parametrize("warps,iters", [(1, 1), (1, 40), (5, 40)])
def test_refine_uniform(warps, iters):
    theta, w_h, w_v = synth.tiny_instance(24, 37, 16, seed=warps * 100 + iters, w_max=0.3)
    labels = np.random.default_rng(1).integers(0, 16, (24, 37))
    err = _refine_case(theta, w_h, w_v, labels, oref.RefineParams(C=3.0, n_warps=warps, n_iters=iters),
                       name=f"uniform-{warps}x{iters}")
    assert err.max() <= U_TOL


@pytest.mark.parametrize("eps,delta", [(1.0, 0.0), (0.5, 0.5), (0.0, 1.0)])
def test_refine_dc_parameters(eps, delta):
    theta, w_h, w_v = synth.tiny_instance(20, 30, 12, seed=7, w_max=0.4)
    labels = np.random.default_rng(2).integers(0, 12, (20, 30))
    err = _refine_case(theta, w_h, w_v, labels, oref.RefineParams(C=2.0, eps=eps, delta=delta, n_warps=2, n_iters=30),
                       name=f"dc-{eps}-{delta}")
    assert err.max() <= U_TOL


def test_refine_stereo_from_dmm_labels_fp16():
    """Stereo-shaped input: SAD cost volume stored in FP16, labels from the oracle's Dual_MM."""
    pair = synth.stereo_pair(80, 48, 24, seed=11, slope=0.08)
    th64 = ocv.sad_cost_volume(pair.left, pair.right, 24)
    w_h, w_v = ocv.contrast_weights(pair.left)
    th16 = th64.astype(np.float16)
    ref = odmm.solve_discrete(th16.astype(np.float64), w_h, w_v, 3, 4)
    err = _refine_case(th16, w_h.astype(np.float32), w_v.astype(np.float32), ref.labels,
                       oref.RefineParams(C=3.0, n_warps=5, n_iters=40), theta_dtype=torch.float16, name="stereo-fp16")
    assert err.max() <= U_TOL


def test_refine_degenerate_shapes():
    for H, W, K in [(1, 9, 5), (9, 1, 5), (1, 1, 3), (4, 4, 1), (3, 5, 2)]:
        theta, w_h, w_v = synth.tiny_instance(H, W, K, seed=H * 10 + W)
        labels = np.random.default_rng(H + W).integers(0, K, (H, W))
        err = _refine_case(theta, w_h, w_v, labels, oref.RefineParams(C=2.0, n_warps=2, n_iters=10),
                           name=f"degenerate-{H}x{W}x{K}")
        assert err.max() <= U_TOL


def test_refine_ragged_tiles():
    """W, H not multiples of the 64 x 4 tile: halo recomputation at every tile border."""
    theta, w_h, w_v = synth.tiny_instance(13, 131, 8, seed=3, w_max=0.5)
    labels = np.random.default_rng(5).integers(0, 8, (13, 131))
    err = _refine_case(theta, w_h, w_v, labels, oref.RefineParams(C=3.0, n_warps=3, n_iters=25), name="ragged")
    assert err.max() <= U_TOL


@pytest.mark.parametrize("window", [1, 3, 5])
def test_cost_volume(window):
    P = _need_gpu()
    pair = synth.stereo_pair(70, 33, 20, seed=window, occlusion_bands=1)
    print(f"[case] cost volume window={window}", flush=True)
    ref = ocv.sad_cost_volume(pair.left, pair.right, 20, window=window, trunc=0.3)
    wh_ref, wv_ref = ocv.contrast_weights(pair.left, 0.1, 0.1)
    L, R = _dev(pair.left), _dev(pair.right)
    c32, wh, wv = P.build_cost_volume(L, R, 20, window=window, dtype=torch.float32)
    c16, _, _ = P.build_cost_volume(L, R, 20, window=window, dtype=torch.float16)
    torch.cuda.synchronize()
    e32 = np.abs(c32.cpu().numpy() - ref).max()
    g16 = c16.cpu().numpy().astype(np.float64)
    r16 = ocv.round_half(ref)
    ulp = np.spacing(np.abs(r16).astype(np.float16)).astype(np.float64)
    e16 = (np.abs(g16 - r16) / ulp).max()
    ew = max(np.abs(wh.cpu().numpy() / wh_ref - 1).max(), np.abs(wv.cpu().numpy() / wv_ref - 1).max())
    print(f"[parity] cost window={window}: f32_abs={e32:.3e} f16_ulps={e16:.2f} w_rel={ew:.3e}", flush=True)
    assert e32 <= 2e-6
    assert e16 <= 1.0
    assert ew <= 1e-6
