"""Parity at the full stereo frame (1242x375, K=192, FP16 cost, 20 dual iterations, T=3,
iterative minorant 1/4, 1/4, 1, the tiles the bench's autotuner picks).

The FP64 oracle cannot run the whole solve within a test's time, so it checks sampled chains
one by one: a horizontal half-step on sampled rows and a vertical half-step on sampled
columns, each from the GPU's own dual before it; the final pass's normalized min-marginals
on sampled rows from the GPU's final dual; and the lower bound (every chain's optimum at the
GPU's final dual).  The backward is checked through properties that hold at any size: the
outputs are positively homogeneous of degree 1 in (cost, weights) (every step of Dual_MM
commutes with scaling), so <cost, dL/dcost> + <w, dL/dw> = L (Euler); a constant added to one
pixel's costs moves LB by that constant and leaves the normalized min-marginals unchanged, so
the per-pixel sums of dL/dcost equal g_lb; and the tape form equals the recomputing form bit
for bit.
"""
import numpy as np
import pytest

import synth
from oracle import chain as och, dmm as odmm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FRAME = dict(W=1242, H=375, K=192, seed=3000, slope=0.08, occlusion_bands=4, segments=16)
T, ITERS, GAMMAS = 3, 20, (0.25, 0.25, 1.0)
ROWS = sorted(set(np.linspace(0, 374, 16).round().astype(int).tolist()))    # 16 rows, both borders included
COLS = sorted(set(np.linspace(0, 1241, 32).round().astype(int).tolist()))   # 32 columns


@pytest.fixture(scope="module")
def frame():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_06274_amd import ops
    W, H, K = FRAME["W"], FRAME["H"], FRAME["K"]
    pair = synth.stereo_pair(W, H, K, seed=FRAME["seed"], segments=FRAME["segments"], slope=FRAME["slope"],
                             occlusion_bands=FRAME["occlusion_bands"])
    dev = torch.device("cuda:0")
    cost, w_h, w_v = ops.build_cost_volume(torch.from_numpy(pair.left).to(dev), torch.from_numpy(pair.right).to(dev),
                                           K, dtype=torch.float16)
    tiles = ops.autotune_tiles((H, W, K), torch.float16, T=T, gammas=GAMMAS)
    torch.cuda.synchronize()
    print(f"[case] full frame {W}x{H}x{K} FP16, tiles {tiles}", flush=True)
    return dict(ops=ops, cost=cost, w_h=w_h, w_v=w_v, kw=dict(T=T, gammas=GAMMAS, tile=tiles),
                th=cost.float().cpu().numpy().astype(np.float64), wh=w_h.cpu().numpy().astype(np.float64),
                wv=w_v.cpu().numpy().astype(np.float64))


def _dual(f, half_steps):
    r = f["ops"].solve_discrete(f["cost"], f["w_h"], f["w_v"], n_half_steps=half_steps, want_minmarg=False,
                                want_bounds=False, **f["kw"])
    return r.dual.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("k", [0, 2 * ITERS - 2])
def test_fullsize_half_steps_sampled(frame, k):
    """One H half-step (16 sampled rows) and the V half-step after it (32 sampled columns)
    against the oracle, from the GPU's dual after k and k + 1 half-steps: the first two
    half-steps of the solve (from the zero dual) and the last two."""
    f = frame
    lam_a = _dual(f, k) if k > 0 else np.zeros(f["th"].shape)
    lam_b, lam_c = _dual(f, k + 1), _dual(f, k + 2)
    scale = max(1.0, np.abs(lam_b).max())
    h = och.iterative_minorant(f["th"][ROWS] - lam_a[ROWS], f["wh"][ROWS], T, GAMMAS)
    err_h = np.abs(lam_a[ROWS] + h - lam_b[ROWS]).max() / scale
    a = np.ascontiguousarray(np.transpose(lam_b[:, COLS], (1, 0, 2)))
    hv = och.iterative_minorant(a, f["wv"][:, COLS].T, T, GAMMAS)
    err_v = np.abs(lam_b[:, COLS] - np.transpose(hv, (1, 0, 2)) - lam_c[:, COLS]).max() / scale
    print(f"[parity] full-size half-steps {k}, {k + 1}: H {err_h:.2e} ({len(ROWS)} rows), V {err_v:.2e} "
          f"({len(COLS)} columns), relative to max |dual| {scale:.3f}", flush=True)
    assert err_h <= 1e-5 and err_v <= 1e-5
    # the other chains moved too (not a no-op)
    assert np.abs(lam_b - lam_a).max() > 1e-3


def test_fullsize_final_pass_and_bound(frame):
    """Final normalized row min-marginals on sampled rows, labels = their argmin everywhere,
    LB against every chain's optimum at the GPU's final dual, LB <= E."""
    f = frame
    ops = f["ops"]
    r = ops.solve_discrete(f["cost"], f["w_h"], f["w_v"], n_iters=ITERS, want_bounds=True, **f["kw"])
    torch.cuda.synchronize()
    lam = r.dual.cpu().numpy().astype(np.float64)
    mm = r.minmarg.cpu().numpy().astype(np.float64)
    labels = r.labels.cpu().numpy()
    th = f["th"]
    S = th.max() - th.min()
    ref = och.min_marginals(th[ROWS] - lam[ROWS], f["wh"][ROWS], T)
    rel = np.abs(mm[ROWS] - ref) / np.maximum(np.abs(ref), S)
    # labels: argmin of the returned min-marginals (lowest label on ties), every pixel
    same = np.array_equal(labels, np.argmin(mm, axis=2))
    lb_gpu, e_gpu = (float(x) for x in r.bounds.cpu().numpy())
    lb_ref = odmm.lower_bound(th, lam, f["wh"], f["wv"], T)
    print(f"[parity] full-size final pass: min-marginal rel {rel.max():.2e}; LB {lb_gpu:.4f} vs {lb_ref:.4f}; "
          f"E {e_gpu:.4f}", flush=True)
    assert rel.max() <= 1e-5
    assert same
    assert abs(lb_gpu - lb_ref) <= 1e-5 * abs(lb_ref)
    assert lb_gpu <= e_gpu + 1e-9 * abs(e_gpu)


def _grads(f, keep, recompute, G_m, g_lb, g_e=0.0, n_iters=ITERS):
    ops = f["ops"]
    r = ops.solve_discrete(f["cost"], f["w_h"], f["w_v"], n_iters=n_iters, want_bounds=True, keep_checkpoints=keep,
                           recompute_selections=recompute, **f["kw"])
    g = ops.solve_discrete_backward(f["cost"], f["w_h"], f["w_v"], r.dual, r.workspace, grad_minmarg=G_m,
                                    grad_lb=g_lb, grad_energy=g_e, n_iters=n_iters, keep_checkpoints=keep,
                                    recompute_selections=recompute, **f["kw"])
    torch.cuda.synchronize()
    out = (r.minmarg.clone(), [float(x) for x in r.bounds.cpu()], [x.clone() for x in g])
    del r, g
    torch.cuda.empty_cache()
    return out


def _backward_properties(f, name, g_lb=0.5, g_e=0.25, seed=11):
    """Euler's identity and the constant-shift identity for L = <G_m, min-marginals> +
    g_lb * LB + g_e * E(labels), with the tapes kept by the forward.  Every output is
    positively homogeneous of degree 1 in (cost, weights), so <cost, dL/dcost> +
    <w, dL/dw> = L; a constant added to one pixel's costs leaves the normalized
    min-marginals unchanged and moves LB and E by that constant, so every pixel's
    dL/dcost sums to g_lb + g_e."""
    gen = torch.Generator(device="cuda").manual_seed(seed)
    G_m = torch.randn(f["cost"].shape, generator=gen, device="cuda", dtype=torch.float32)
    mm, (lb, e), (gc, gwh, gwv) = _grads(f, 2, False, G_m, g_lb, g_e)
    L = float((G_m.double() * mm.double()).sum()) + g_lb * lb + g_e * e
    euler = float((f["cost"].double() * gc.double()).sum() + (f["w_h"].double() * gwh.double()).sum()
                  + (f["w_v"].double() * gwv.double()).sum())
    scale = float((f["cost"].double() * gc.double()).abs().sum() + (f["w_h"].double() * gwh.double()).abs().sum()
                  + (f["w_v"].double() * gwv.double()).abs().sum())
    shift = (gc.double().sum(dim=2) - (g_lb + g_e)).abs().max().item()
    print(f"[parity] {name} backward: Euler {euler:.6f} vs L {L:.6f} (scale {scale:.1f}); per-pixel sum of "
          f"dL/dcost - (g_lb + g_e): max {shift:.2e}", flush=True)
    assert abs(euler - L) <= 1e-5 * scale
    assert shift <= 1e-3
    assert torch.isfinite(gc).all() and torch.isfinite(gwh).all() and torch.isfinite(gwv).all()


def test_fullsize_backward_properties(frame):
    """The identities at the bench frame (1242x375x192, FP16 cost)."""
    _backward_properties(frame, "full-size")


def test_differentiation_frame_backward_properties():
    """The identities at the differentiation workload's frame size (960x320, K=96, FP32 cost,
    20 dual iterations, the tapes kept by the forward)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_06274_amd import ops
    W, H, K = 960, 320, 96
    pair = synth.stereo_pair(W, H, K, seed=5000, slope=0.08, occlusion_bands=2)
    dev = torch.device("cuda:0")
    print(f"[case] differentiation frame {W}x{H}x{K} FP32", flush=True)
    cost, w_h, w_v = ops.build_cost_volume(torch.from_numpy(pair.left).to(dev), torch.from_numpy(pair.right).to(dev),
                                           K, dtype=torch.float32)
    f = dict(ops=ops, cost=cost, w_h=w_h, w_v=w_v, kw=dict(T=T, gammas=GAMMAS))
    _backward_properties(f, "960x320x96", seed=13)


def test_fullsize_tape_equals_recompute(frame):
    """The backward from forward-kept tapes equals the backward that recomputes every
    half-step and every selection (window search) bit for bit at the full frame."""
    f = frame
    gen = torch.Generator(device="cuda").manual_seed(12)
    G_m = torch.randn(f["cost"].shape, generator=gen, device="cuda", dtype=torch.float32)
    _, _, g_tape = _grads(f, 2, False, G_m, 1.0)
    _, _, g_rec = _grads(f, 1, True, G_m, 1.0)
    for a, b in zip(g_tape, g_rec):
        assert torch.equal(a, b), float((a - b).abs().max())


def test_config_640x480_fp32_with_refinement():
    """The 640x480, K=128 stereo workload (FP32 cost, 20 dual iterations, then refinement
    5 warps x 40 iterations): the whole cost volume, the final min-marginals of sampled rows
    and the lower bound from the GPU's final dual, and the whole refinement from the GPU's
    labels, against the oracle."""
    from oracle import cost_volume as ocv, refine as oref
    from paper_1601_06274_amd import ops
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    W, H, K = 640, 480, 128
    pair = synth.stereo_pair(W, H, K, seed=2000, segments=12, slope=0.02)
    dev = torch.device("cuda:0")
    print(f"[case] stereo {W}x{H}x{K} FP32 + refinement", flush=True)
    cost, w_h, w_v = ops.build_cost_volume(torch.from_numpy(pair.left).to(dev),
                                           torch.from_numpy(pair.right).to(dev), K, dtype=torch.float32)
    r = ops.solve_discrete(cost, w_h, w_v, T=T, n_iters=ITERS, gammas=GAMMAS, want_bounds=True)
    u = ops.refine_continuous(cost, r.labels, w_h, w_v, C=3.0, n_warps=5, n_iters=40)
    torch.cuda.synchronize()
    th = cost.cpu().numpy().astype(np.float64)
    wh, wv = w_h.cpu().numpy().astype(np.float64), w_v.cpu().numpy().astype(np.float64)
    err_cv = np.abs(th - ocv.sad_cost_volume(pair.left, pair.right, K)).max()
    lam = r.dual.cpu().numpy().astype(np.float64)
    mm = r.minmarg.cpu().numpy().astype(np.float64)
    rows = [0, 239, 479]
    ref = och.min_marginals(th[rows] - lam[rows], wh[rows], T)
    S = th.max() - th.min()
    rel = (np.abs(mm[rows] - ref) / np.maximum(np.abs(ref), S)).max()
    lb_gpu = float(r.bounds[0])
    lb_ref = odmm.lower_bound(th, lam, wh, wv, T)
    labels = r.labels.cpu().numpy()
    f32 = lambda v: float(np.float32(v))  # the C ABI takes float32 parameters
    u_ref = oref.refine_continuous(th, wh, wv, labels, oref.RefineParams(C=3.0, tau=f32(0.3), sigma=f32(0.3),
                                                                          n_warps=5, n_iters=40))
    err_u = np.abs(u.cpu().numpy() - u_ref).max()
    print(f"[parity] 640x480: cost volume {err_cv:.2e}, min-marginals rel {rel:.2e}, LB {lb_gpu:.4f} vs "
          f"{lb_ref:.4f}, refined u {err_u:.2e}", flush=True)
    assert err_cv <= 2e-6
    assert rel <= 1e-5
    assert abs(lb_gpu - lb_ref) <= 1e-5 * abs(lb_ref)
    assert np.array_equal(labels, np.argmin(mm, axis=2))
    assert err_u <= 1e-4


def test_fullsize_refinement(frame):
    """Refinement at the full frame (FP16 cost, 5 warps x 40 iterations, C = 3) from the
    GPU's labels, against the oracle on the same labels."""
    from oracle import refine as oref
    f = frame
    ops = f["ops"]
    r = ops.solve_discrete(f["cost"], f["w_h"], f["w_v"], n_iters=ITERS, want_minmarg=False, want_bounds=False,
                           **f["kw"])
    u = ops.refine_continuous(f["cost"], r.labels, f["w_h"], f["w_v"], C=3.0, n_warps=5, n_iters=40)
    torch.cuda.synchronize()
    f32 = lambda v: float(np.float32(v))  # the C ABI takes float32 parameters
    u_ref = oref.refine_continuous(f["th"], f["wh"], f["wv"], r.labels.cpu().numpy(),
                                   oref.RefineParams(C=3.0, tau=f32(0.3), sigma=f32(0.3), n_warps=5, n_iters=40))
    err = np.abs(u.cpu().numpy() - u_ref).max()
    print(f"[parity] full-size refinement: max |u - u_ref| {err:.2e}", flush=True)
    assert err <= 1e-4
