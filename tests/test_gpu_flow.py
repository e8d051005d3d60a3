"""GPU parity of the optical-flow entry points against the FP64 oracle (Sec. 2.2 "Flow",
Sec. 3.2): the two-dimensional SAD cost (FP32 within 2e-6, FP16 within one half-precision
ulp of the oracle's value), the decoupled layer costs (bit-exact: minima of the same
values), the quadratic-fit refinement (|du| <= 1e-4 from the same labels), and the whole
pipeline on a synthetic pair."""
import numpy as np
import pytest

import synth
from oracle import cost_volume as ocv, flow as oflow
from oracle.refine import RefineParams

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_06274_amd import ops
    return ops


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _f32(v):
    return float(np.float32(v))


@pytest.mark.parametrize("W,H,K1,K2,off1,off2,window,dtype", [
    (70, 9, 5, 3, 2, 1, 3, torch.float32),
    (130, 7, 17, 9, 8, 4, 3, torch.float16),
    (40, 12, 32, 32, 16, 16, 3, torch.float32),
    (64, 5, 3, 7, 0, 6, 5, torch.float32),
    (1, 1, 4, 4, 2, 2, 3, torch.float32),
    (33, 3, 1, 1, 0, 0, 1, torch.float16),
])
def test_flow_cost_volume(W, H, K1, K2, off1, off2, window, dtype):
    ops = _need()
    pair = synth.flow_pair(W, H, 3.0, seed=W + H + K1, segments=2)
    print(f"[case] flow cost {W}x{H} K1={K1} K2={K2} off=({off1},{off2}) window={window} {dtype}", flush=True)
    cost, w_h, w_v = ops.build_flow_cost_volume(_dev(pair.first), _dev(pair.second), K1, K2, off1, off2,
                                                window=window, dtype=dtype)
    torch.cuda.synchronize()
    ref = oflow.flow_cost_volume(pair.first, pair.second, K1, K2, off1, off2, window=window, trunc=_f32(0.3))
    got = cost.float().cpu().numpy().astype(np.float64)
    if dtype == torch.float32:
        err = np.abs(got - ref).max()
        assert err <= 2e-6, err
    else:
        # within one half-precision ulp of the oracle's value rounded to half
        r16 = ocv.round_half(ref)
        ulp = np.spacing(np.abs(r16).astype(np.float16)).astype(np.float64)
        assert np.all(np.abs(got - r16) <= ulp), np.abs(got - r16).max()
    wh_ref, wv_ref = ocv.contrast_weights(pair.first)
    assert np.abs(w_h.cpu().numpy() - wh_ref).max(initial=0.0) <= 1e-6
    assert np.abs(w_v.cpu().numpy() - wv_ref).max(initial=0.0) <= 1e-6


@pytest.mark.parametrize("K1,K2,dtype", [(1, 1, torch.float32), (3, 5, torch.float16), (32, 32, torch.float32),
                                         (64, 64, torch.float16), (256, 16, torch.float32), (16, 256, torch.float16),
                                         (65, 63, torch.float32)])
def test_flow_project_bitexact(K1, K2, dtype):
    ops = _need()
    H, W = 5, 13
    g = np.random.default_rng(K1 * 7 + K2)
    D = g.random((H, W, K2, K1))
    D[0, 0] = 0.25                      # a pixel whose every entry ties
    cost = _dev(D, dtype)
    print(f"[case] flow projection K1={K1} K2={K2} {dtype}", flush=True)
    f1, f2 = ops.flow_project(cost)
    torch.cuda.synchronize()
    r1, r2 = oflow.project(cost.float().cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(f1.float().cpu().numpy(), r1)
    np.testing.assert_array_equal(f2.float().cpu().numpy(), r2)


@pytest.mark.parametrize("H,W,K1,K2,warps,iters,C,dtype", [
    (6, 9, 7, 5, 2, 15, 2.0, torch.float32),
    (13, 70, 9, 9, 3, 10, 3.0, torch.float16),
    (1, 20, 5, 4, 1, 30, 2.0, torch.float32),
    (9, 1, 4, 6, 2, 10, 2.0, torch.float32),
])
def test_flow_refine_parity(H, W, K1, K2, warps, iters, C, dtype):
    """Both components from the same labels, against the oracle: |du| <= 1e-4."""
    ops = _need()
    g = np.random.default_rng(H * W + K1)
    D = g.random((H, W, K2, K1))
    w_h = (g.random((H, max(W - 1, 0))) * 0.5).astype(np.float32)
    w_v = (g.random((max(H - 1, 0), W)) * 0.5).astype(np.float32)
    l1 = g.integers(0, K1, (H, W))
    l2 = g.integers(0, K2, (H, W))
    cost = _dev(D, dtype)
    print(f"[case] flow refine {H}x{W} K1={K1} K2={K2} {warps}x{iters} {dtype}", flush=True)
    u1, u2 = ops.refine_flow(cost, _dev(l1, torch.int32), _dev(l2, torch.int32), _dev(w_h), _dev(w_v), C=C,
                             n_warps=warps, n_iters=iters)
    torch.cuda.synchronize()
    P = RefineParams(C=C, tau=_f32(0.3), sigma=_f32(0.3), n_warps=warps, n_iters=iters)
    r1, r2 = oflow.refine_flow(cost.float().cpu().numpy().astype(np.float64), w_h, w_v, l1, l2, P)
    err = max(np.abs(u1.cpu().numpy() - r1).max(), np.abs(u2.cpu().numpy() - r2).max())
    print(f"[parity] flow refine: max |du| {err:.2e}", flush=True)
    assert err <= 1e-4


def test_flow_pipeline_synthetic_pair():
    """Cost volume, decoupled costs, two Dual_MM solves and the refinement on a synthetic
    160 x 96 pair with displacements up to 7 px (K1 = K2 = 16): the layer labels equal the
    oracle's up to exact-cost ties, the refinement from the oracle's labels matches within
    1e-4, and the recovered flow is within a pixel of the truth on most pixels."""
    ops = _need()
    W, H, R = 160, 96, 8
    K = 2 * R
    pair = synth.flow_pair(W, H, R - 1.0, seed=61, segments=4, slope=0.01)
    print(f"[case] flow pipeline {W}x{H} K={K}", flush=True)
    cost, w_h, w_v = ops.build_flow_cost_volume(_dev(pair.first), _dev(pair.second), K, K, R, R, lambda_pw=0.05)
    res = ops.solve_flow(cost, w_h, w_v, off1=R, off2=R, T=3, n_iters=10, refine=False)
    torch.cuda.synchronize()
    D = cost.cpu().numpy().astype(np.float64)
    wh, wv = w_h.cpu().numpy().astype(np.float64), w_v.cpu().numpy().astype(np.float64)
    ref = oflow.solve_flow(D, wh, wv, 3, 10, RefineParams(C=3.0, n_warps=0, n_iters=0))
    from tests.parity import check_labels, minmarg_errors
    for layer, rl, f_ref in ((res.layer1, ref.layer1, ref.f1), (res.layer2, ref.layer2, ref.f2)):
        _, rel = minmarg_errors(layer.minmarg.cpu().numpy(), rl.minmarg, f_ref)
        ndiff, nbad = check_labels(layer.labels.cpu().numpy(), rl.labels, rl.minmarg, f_ref)
        print(f"[parity] flow layer: min-marginal rel {rel.max():.2e}, label diffs {ndiff} (non-ties {nbad})",
              flush=True)
        assert rel.max() <= 1e-5 and nbad == 0
    l1, l2 = ref.layer1.labels, ref.layer2.labels
    u1, u2 = ops.refine_flow(cost, _dev(l1, torch.int32), _dev(l2, torch.int32), w_h, w_v, off1=R, off2=R, C=3.0,
                             n_warps=3, n_iters=20)
    torch.cuda.synchronize()
    P = RefineParams(C=3.0, tau=_f32(0.3), sigma=_f32(0.3), n_warps=3, n_iters=20)
    r1, r2 = oflow.refine_flow(D, wh, wv, l1, l2, P)
    err = max(np.abs(u1.cpu().numpy() - r1).max(), np.abs(u2.cpu().numpy() - r2).max())
    flow_err = np.hypot(u1.cpu().numpy() - R - pair.flow[..., 0], u2.cpu().numpy() - R - pair.flow[..., 1])[4:-4, 4:-4]
    print(f"[parity] flow pipeline: refined |du| {err:.2e}; flow error median {np.median(flow_err):.3f} px, "
          f"{np.mean(flow_err < 1):.3f} within 1 px", flush=True)
    assert err <= 1e-4
    assert np.median(flow_err) < 0.5 and np.mean(flow_err < 1.0) > 0.7


def test_flow_full_frame_sampled():
    """The paper's flow frame size, 640 x 480, displacements -16..15 in both directions
    (K1 = K2 = 32, FP16 cost): the cost volume on sampled rows against the oracle on a band
    of rows around them, the decoupled costs at every pixel of those rows (bit-exact), and
    the refinement of both components at every pixel from the same labels (5 x 40)."""
    ops = _need()
    W, H, R = 640, 480, 16
    K = 2 * R
    pair = synth.flow_pair(W, H, 12.0, seed=62, slope=0.01)
    print(f"[case] flow full frame {W}x{H} K={K} FP16", flush=True)
    cost, w_h, w_v = ops.build_flow_cost_volume(_dev(pair.first), _dev(pair.second), K, K, R, R,
                                                dtype=torch.float16)
    f1, f2 = ops.flow_project(cost)
    torch.cuda.synchronize()
    # rows 0, 240 and 479 (the oracle evaluates only those output rows)
    for y in (0, 240, 479):
        D_ref = oflow.flow_cost_volume(pair.first, pair.second, K, K, R, R, trunc=_f32(0.3), rows=(y, y + 1))[0]
        got = cost[y].float().cpu().numpy().astype(np.float64)
        r16 = ocv.round_half(D_ref)
        ulp = np.spacing(np.abs(r16).astype(np.float16)).astype(np.float64)
        assert np.all(np.abs(got - r16) <= ulp), (y, np.abs(got - r16).max())
        e1, e2 = oflow.project(got[None])
        assert np.array_equal(f1[y].float().cpu().numpy(), e1[0]) and np.array_equal(f2[y].float().cpu().numpy(), e2[0])
    g = np.random.default_rng(5)
    l1 = g.integers(0, K, (H, W))
    l2 = g.integers(0, K, (H, W))
    u1, u2 = ops.refine_flow(cost, _dev(l1, torch.int32), _dev(l2, torch.int32), w_h, w_v, off1=R, off2=R, C=3.0,
                             n_warps=5, n_iters=40)
    torch.cuda.synchronize()
    D = cost.float().cpu().numpy().astype(np.float64)
    P = RefineParams(C=3.0, tau=_f32(0.3), sigma=_f32(0.3), n_warps=5, n_iters=40)
    r1, r2 = oflow.refine_flow(D, w_h.cpu().numpy().astype(np.float64), w_v.cpu().numpy().astype(np.float64), l1, l2, P)
    err = max(np.abs(u1.cpu().numpy() - r1).max(), np.abs(u2.cpu().numpy() - r2).max())
    print(f"[parity] flow full frame: refined |du| {err:.2e}", flush=True)
    assert err <= 1e-4


def test_flow_layers_on_two_streams_equal_one_stream():
    """The second layer's solve on a forked stream gives the one-stream results bit for bit
    (labels, min-marginals, duals, bounds and the refined flow), on three calls in a row."""
    ops = _need()
    W, H, R = 200, 120, 8
    K = 2 * R
    pair = synth.flow_pair(W, H, R - 1.0, seed=63, segments=5, slope=0.01)
    print(f"[case] flow two streams {W}x{H} K={K}", flush=True)
    cost, w_h, w_v = ops.build_flow_cost_volume(_dev(pair.first), _dev(pair.second), K, K, R, R,
                                                dtype=torch.float16)
    ref = ops.solve_flow(cost, w_h, w_v, off1=R, off2=R, T=3, n_iters=6, two_streams=False,
                         refine=dict(C=3.0, n_warps=2, n_iters=10))
    torch.cuda.synchronize()
    for rep in range(3):
        got = ops.solve_flow(cost, w_h, w_v, off1=R, off2=R, T=3, n_iters=6, two_streams=True,
                             refine=dict(C=3.0, n_warps=2, n_iters=10))
        torch.cuda.synchronize()
        for a, b in ((got.layer1, ref.layer1), (got.layer2, ref.layer2)):
            assert torch.equal(a.labels, b.labels), f"call {rep}: labels"
            assert torch.equal(a.minmarg, b.minmarg), f"call {rep}: min-marginals"
            assert torch.equal(a.dual, b.dual), f"call {rep}: duals"
            assert torch.equal(a.bounds, b.bounds), f"call {rep}: bounds"
        assert torch.equal(got.u1, ref.u1) and torch.equal(got.u2, ref.u2), f"call {rep}: refined flow"
