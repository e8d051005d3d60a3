"""GPU parity of dm_solve_discrete against the FP64 oracle (Dual_MM, Sec. 2.3).

Acceptance (float32 state on the GPU, float64 oracle):
  * labels identical except at exact-cost ties within the min-marginal tolerance;
  * normalized min-marginals |gpu - ref| <= 1e-5 * max(|ref|, S), S = cost range;
  * lower bound and energy: relative 1e-5 (bound) and 1e-9 (energy, FP64 sums of the
    same float32 inputs); the bound never exceeds the energy; the bound trace
    never decreases by more than the float32 noise of the sums.
"""
import numpy as np
import pytest

import synth
from oracle import dmm as odmm, energy as oenergy, cost_volume as ocv
from paper_1601_06274_amd.build import TILES  # the compiled tile list (read from csrc/tiles.h)
from tests.parity import MM_RTOL, check_labels, minmarg_errors, summarize

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_06274_amd import solve_discrete
    return solve_discrete


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _run_both(theta, w_h, w_v, T, n_iters, *, minorant="iterative", gammas=(0.25, 0.25, 1.0), half_steps=0,
              theta_dtype=torch.float32, tile=None, name=""):
    solve = _gpu()
    print(f"[case] {name} shape={theta.shape} T={T} iters={n_iters} half={half_steps} {minorant} "
          f"{theta_dtype} tile={tile}", flush=True)
    th_dev = _dev(theta, theta_dtype)
    theta_used = th_dev.float().cpu().numpy().astype(np.float64)   # exactly what the GPU reads
    res = solve(th_dev, _dev(w_h), _dev(w_v), T=T, n_iters=n_iters, n_half_steps=half_steps, minorant=minorant,
                gammas=gammas, want_trace=True, tile=tile)
    torch.cuda.synchronize()
    ref = odmm.solve_discrete(theta_used, w_h.astype(np.float64), w_v.astype(np.float64), T, n_iters,
                              minorant=minorant, gammas=gammas, n_half_steps=half_steps or None)
    return res, ref, theta_used


def _check(res, ref, theta_used, w_h, w_v, T, name):
    mm = res.minmarg.cpu().numpy()
    err, rel = minmarg_errors(mm, ref.minmarg, theta_used)
    lab = res.labels.cpu().numpy()
    ndiff, nbad = check_labels(lab, ref.labels, ref.minmarg, theta_used)
    b = res.bounds.cpu().numpy()
    tr = res.lb_trace.cpu().numpy()
    e_lab = oenergy.grid_energy(theta_used, w_h, w_v, T, lab)
    summarize(name, mm_abs=float(err.max()), mm_rel=float(rel.max()), label_diff=ndiff, label_bad=nbad,
              lb_gpu=float(b[0]), lb_ref=ref.lower_bound, e_gpu=float(b[1]), e_ref=ref.energy,
              trace_err=float(np.abs(tr - ref.lb_trace).max()) if len(tr) else 0.0,
              lam_err=float(np.abs(res.dual.cpu().numpy() - ref.lam).max()))
    assert rel.max() <= MM_RTOL, f"min-marginal rel err {rel.max():.3e}"
    assert nbad == 0, f"{nbad} label mismatches that are not ties"
    # the dual state itself, with the min-marginals' bar
    lam = res.dual.cpu().numpy().astype(np.float64)
    S = max(float(theta_used.max() - theta_used.min()), 1e-12)
    lam_rel = np.abs(lam - ref.lam) / np.maximum(np.abs(ref.lam), S)
    assert lam_rel.max() <= MM_RTOL, f"dual rel err {lam_rel.max():.3e}"
    assert b[1] == pytest.approx(e_lab, rel=1e-9, abs=1e-9)
    scale = max(abs(ref.lower_bound), 1.0)
    assert abs(b[0] - ref.lower_bound) <= 1e-5 * scale
    assert b[0] <= b[1] + 1e-6 * scale
    np.testing.assert_allclose(tr, ref.lb_trace, rtol=0, atol=1e-5 * scale)


def test_config1_uniform_128x96_k32():
    """128x96 grid, K=32, U[0,1) unaries (seed 0), w=0.1, T=3, 10 dual iterations."""
    theta, w_h, w_v = synth.uniform_unaries(96, 128, 32, seed=0, w=0.1)
    res, ref, th = _run_both(theta, w_h, w_v, 3, 10, name="config1")
    _check(res, ref, th, w_h, w_v, 3, "config1")


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8, 13, 17, 32, 48, 64, 96, 100, 128, 160, 192, 256])
def test_label_counts_and_tiles(K):
    """Every tile path (exact and partial) on a small grid with ragged label counts."""
    H, W = 7, 11
    theta, w_h, w_v = synth.tiny_instance(H, W, K, seed=K, w_max=0.3)
    res, ref, th = _run_both(theta, w_h, w_v, 2 if K > 1 else 1, 3, name=f"K{K}")
    _check(res, ref, th, w_h, w_v, 2 if K > 1 else 1, f"K{K}")


@pytest.mark.parametrize("tile", TILES)
def test_forced_tiles_full(tile):
    """Every compiled tile with K = lanes x labels per lane (vector loads, no masked labels)."""
    K = tile[0] * tile[1]
    theta, w_h, w_v = synth.tiny_instance(5, 7, K, seed=100 + K, w_max=0.4)
    res, ref, th = _run_both(theta, w_h, w_v, 3, 2, tile=tile, name=f"full{tile}")
    _check(res, ref, th, w_h, w_v, 3, f"full{tile}")
    res, ref, th = _run_both(theta.astype(np.float16), w_h, w_v, 3, 2, theta_dtype=torch.float16, tile=tile,
                             name=f"full16{tile}")
    _check(res, ref, th, w_h, w_v, 3, f"full16{tile}")


@pytest.mark.parametrize("tile", TILES)
def test_forced_tiles(tile):
    K = min(tile[0] * tile[1], 24)
    theta, w_h, w_v = synth.tiny_instance(9, 13, K, seed=100 + K, w_max=0.4)
    res, ref, th = _run_both(theta, w_h, w_v, 3, 2, tile=tile, name=f"tile{tile}")
    _check(res, ref, th, w_h, w_v, 3, f"tile{tile}")


@pytest.mark.parametrize("T", [1, 2, 4, 7, 40])
def test_truncations(T):
    """Distance-transform reach across lanes: T-1 spans 0, 1, 2 and all lanes."""
    theta, w_h, w_v = synth.tiny_instance(6, 10, 20, seed=T, w_max=0.2)
    res, ref, th = _run_both(theta, w_h, w_v, T, 2, tile=(8, 4) if T < 10 else None, name=f"T{T}")
    _check(res, ref, th, w_h, w_v, T, f"T{T}")
    res2, ref2, th2 = _run_both(theta, w_h, w_v, T, 2, tile=(32, 3), name=f"T{T}-32x3")
    _check(res2, ref2, th2, w_h, w_v, T, f"T{T}-32x3")


@pytest.mark.parametrize("half", [1, 2, 3, 5])
def test_odd_half_steps(half):
    theta, w_h, w_v = synth.tiny_instance(8, 9, 6, seed=half, w_max=0.5)
    res, ref, th = _run_both(theta, w_h, w_v, 2, 0, half_steps=half, name=f"half{half}")
    _check(res, ref, th, w_h, w_v, 2, f"half{half}")


def test_zero_iterations_bounds():
    theta, w_h, w_v = synth.tiny_instance(5, 6, 4, seed=1)
    solve = _gpu()
    res = solve(_dev(theta), _dev(w_h), _dev(w_v), T=2, n_iters=0)
    ref = odmm.solve_discrete(theta.astype(np.float64), w_h, w_v, 2, 0)
    b = res.bounds.cpu().numpy()
    assert b[0] == pytest.approx(ref.lower_bound, abs=1e-5)
    assert b[1] == pytest.approx(ref.energy, abs=1e-6)


def test_naive_minorant():
    theta, w_h, w_v = synth.tiny_instance(10, 12, 8, seed=3, w_max=0.5)
    res, ref, th = _run_both(theta, w_h, w_v, 2, 4, minorant="naive", name="naive")
    _check(res, ref, th, w_h, w_v, 2, "naive")


@pytest.mark.parametrize("gammas", [(1.0,), (0.5, 1.0), (0.25, 0.25, 0.25, 0.25, 0.25, 1.0)])
def test_gamma_schedules(gammas):
    theta, w_h, w_v = synth.tiny_instance(8, 10, 12, seed=len(gammas), w_max=0.4)
    res, ref, th = _run_both(theta, w_h, w_v, 3, 3, gammas=gammas, name=f"gammas{len(gammas)}")
    _check(res, ref, th, w_h, w_v, 3, f"gammas{len(gammas)}")


@pytest.mark.parametrize("seed", range(20))
def test_bruteforce_3x3(seed):
    """3x3 grids, K=3: GPU LB <= exact minimum <= energy of the GPU labels; oracle parity."""
    T = 1 + seed % 2
    theta, w_h, w_v = synth.tiny_instance(3, 3, 3, seed=seed)
    res, ref, th = _run_both(theta, w_h, w_v, T, 3, name=f"bf{seed}")
    emin, _ = oenergy.brute_force_min(th, w_h, w_v, T)
    b = res.bounds.cpu().numpy()
    assert b[0] <= emin + 1e-6
    assert b[1] >= emin - 1e-9
    _check(res, ref, th, w_h, w_v, T, f"bf{seed}")


def test_fp16_cost_storage():
    """FP16 cost volume: parity against the oracle run on the rounded values."""
    pair = synth.stereo_pair(96, 40, 32, seed=7)
    th64 = ocv.sad_cost_volume(pair.left, pair.right, 32)
    w_h, w_v = ocv.contrast_weights(pair.left)
    w_h = w_h.astype(np.float32)
    w_v = w_v.astype(np.float32)
    res, ref, th = _run_both(th64.astype(np.float16), w_h, w_v, 3, 4, theta_dtype=torch.float16, name="fp16")
    np.testing.assert_array_equal(th, ocv.round_half(th64))
    _check(res, ref, th, w_h, w_v, 3, "fp16")
    # energy error of FP16 storage: the GPU labeling scored on the unrounded costs against
    # the FP64 oracle's own labeling of the unrounded problem
    ref64 = odmm.solve_discrete(th64, w_h.astype(np.float64), w_v.astype(np.float64), 3, 4)
    e16 = oenergy.grid_energy(th64, w_h, w_v, 3, res.labels.cpu().numpy())
    e64 = oenergy.grid_energy(th64, w_h, w_v, 3, ref64.labels)
    rel = (e16 - e64) / e64
    print(f"[parity] fp16 storage energy error vs fp64: E16={e16:.6f} E64={e64:.6f} rel={rel:.3e}", flush=True)
    assert abs(rel) <= 5e-3


def test_warm_start_resume():
    """5 + 5 iterations with the dual carried over equals 10 iterations (same kernels, same order)."""
    solve = _gpu()
    theta, w_h, w_v = synth.tiny_instance(12, 16, 16, seed=5, w_max=0.4)
    th, wh, wv = _dev(theta), _dev(w_h), _dev(w_v)
    a = solve(th, wh, wv, T=3, n_iters=5)
    b = solve(th, wh, wv, T=3, n_iters=5, dual=a.dual.clone(), warm_start=True)
    c = solve(th, wh, wv, T=3, n_iters=10)
    torch.cuda.synchronize()
    assert torch.equal(b.dual, c.dual)
    assert torch.equal(b.labels, c.labels)


def test_deterministic():
    solve = _gpu()
    theta, w_h, w_v = synth.uniform_unaries(40, 50, 32, seed=2)
    th, wh, wv = _dev(theta), _dev(w_h), _dev(w_v)
    a = solve(th, wh, wv, T=3, n_iters=3)
    b = solve(th, wh, wv, T=3, n_iters=3)
    torch.cuda.synchronize()
    assert torch.equal(a.dual, b.dual) and torch.equal(a.minmarg, b.minmarg) and torch.equal(a.bounds, b.bounds)
