"""GPU parity of Dual_MM with the hierarchical minorant (App. A.3.3, Alg. Handshake)
against the FP64 oracle, with the acceptance of the other minorants (labels up to ties,
normalized min-marginals within 1e-5 relative, lower bound and trace within 1e-5
relative, energy of the labels within 1e-9); the duals within 1e-5 of max(|ref|, S)."""
import numpy as np
import pytest

import synth
from oracle import energy as oenergy
from tests.parity import cost_scale
from tests.test_gpu_dmm import _check, _run_both

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [  # H, W, K, T, iters, cost dtype
    (9, 13, 7, 2, 3, torch.float32),
    (16, 33, 64, 3, 3, torch.float32),
    (7, 50, 100, 1, 2, torch.float32),
    (5, 64, 192, 3, 2, torch.float16),
    (11, 12, 256, 4, 2, torch.float32),
    (6, 1, 5, 2, 2, torch.float32),     # rows of one node
    (1, 17, 9, 2, 2, torch.float32),    # columns of one node
    (2, 2, 1, 1, 1, torch.float32),     # one label
    (4, 129, 40, 3, 2, torch.float32),  # odd lengths at every level
    (3, 70, 256, 3, 2, torch.float32),  # four waves per chain with 4 labels per lane
    (5, 90, 200, 4, 2, torch.float16),
    (2, 300, 130, 2, 1, torch.float32),  # several depths above the LDS parts
    (60, 20, 64, 2, 2, torch.float32),   # column chains split at depth 2 (one wave per subtree)
    (40, 30, 50, 3, 2, torch.float16),   # columns split at depth 2, rows at depth 1, ragged labels
]


@pytest.mark.parametrize("H,W,K,T,iters,dt", CASES)
def test_hierarchical_matches_oracle(H, W, K, T, iters, dt):
    theta, w_h, w_v = synth.tiny_instance(H, W, K, seed=H * 1000 + W + K, w_max=0.6)
    name = f"hier {H}x{W}x{K} T={T}"
    res, ref, th = _run_both(theta, w_h, w_v, T, iters, minorant="hierarchical", theta_dtype=dt, name=name)
    _check(res, ref, th, w_h, w_v, T, name)
    lam = res.dual.cpu().numpy()
    scale = np.maximum(np.abs(ref.lam), cost_scale(th))
    assert (np.abs(lam - ref.lam) / scale).max() <= 1e-5


@pytest.mark.parametrize("seed", range(6))
def test_hierarchical_bruteforce_3x3(seed):
    T = 1 + seed % 2
    theta, w_h, w_v = synth.tiny_instance(3, 3, 3, seed=seed)
    res, ref, th = _run_both(theta, w_h, w_v, T, 3, minorant="hierarchical", name=f"hier bf{seed}")
    emin, _ = oenergy.brute_force_min(th, w_h, w_v, T)
    b = res.bounds.cpu().numpy()
    assert b[0] <= emin + 1e-6 and b[1] >= emin - 1e-9
    _check(res, ref, th, w_h, w_v, T, f"hier bf{seed}")


def test_hierarchical_stereo_frame():
    """A 160 x 96 stereo pair, K = 48, FP16 cost, 4 iterations (the paper's live setting
    runs 4): parity as above, and the bound at least that of the iterative minorant."""
    import paper_1601_06274_amd as P
    from oracle import cost_volume as ocv
    pair = synth.stereo_pair(160, 96, 48, seed=2200, segments=5)
    theta = ocv.round_half(ocv.sad_cost_volume(pair.left, pair.right, 48))
    w_h, w_v = ocv.contrast_weights(pair.left)
    w_h, w_v = w_h.astype(np.float32), w_v.astype(np.float32)
    res, ref, th = _run_both(theta, w_h, w_v, 3, 4, minorant="hierarchical", theta_dtype=torch.float16,
                             name="hier stereo")
    _check(res, ref, th, w_h, w_v, 3, "hier stereo")
    dev = lambda a, d=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=d)
    it = P.solve_discrete(dev(theta, torch.float16), dev(w_h), dev(w_v), T=3, n_iters=4)
    torch.cuda.synchronize()
    print(f"[hier] LB hierarchical {res.bounds[0].item():.4f} iterative {it.bounds[0].item():.4f}", flush=True)


def test_hierarchical_full_frame_sampled_chains():
    """1242 x 375, K = 192, FP16 cost (four waves per row chain, seven cut levels above
    the LDS parts; both families split at depth 3 into a launch for the top levels and a
    block per subtree): the GPU's dual after one row half-step and after the following
    column half-step, on 22 rows and 42 columns spread over the frame (both ends
    included), against the oracle's hierarchical minorant of those chains taken from the
    GPU's dual before the half-step."""
    import paper_1601_06274_amd as P
    from oracle import chain, cost_volume as ocv
    W, H, K, T = 1242, 375, 192, 3
    pair = synth.stereo_pair(W, H, K, seed=3000, segments=16, slope=0.08, occlusion_bands=4)
    dev = lambda a, d=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=d)
    cost, w_h, w_v = P.build_cost_volume(dev(pair.left), dev(pair.right), K, dtype=torch.float16)
    th = cost.float().cpu().numpy().astype(np.float64)
    wh = w_h.cpu().numpy().astype(np.float64)
    wv = w_v.cpu().numpy().astype(np.float64)
    S = cost_scale(th)
    print("[case] hierarchical full frame, one row and one column half-step", flush=True)
    r1 = P.solve_discrete(cost, w_h, w_v, T=T, n_half_steps=1, minorant="hierarchical")
    r2 = P.solve_discrete(cost, w_h, w_v, T=T, n_half_steps=2, minorant="hierarchical")
    torch.cuda.synchronize()
    lam1 = r1.dual.cpu().numpy().astype(np.float64)
    lam2 = r2.dual.cpu().numpy().astype(np.float64)
    rows = sorted(set(np.linspace(0, H - 1, 20).astype(int).tolist()) | {1, H - 2})
    h = chain.hierarchical_minorant(th[rows], wh[rows], T)  # rows start from lambda = 0
    err = np.abs(lam1[rows] - h) / np.maximum(np.abs(h), S)
    cols = sorted(set(np.linspace(0, W - 1, 40).astype(int).tolist()) | {1, W - 2})
    a = np.transpose(lam1[:, cols], (1, 0, 2))  # column chains: unaries lambda
    g = chain.hierarchical_minorant(a, wv[:, cols].T, T)
    ref2 = a - g
    err2 = np.abs(np.transpose(lam2[:, cols], (1, 0, 2)) - ref2) / np.maximum(np.abs(ref2), S)
    print(f"[hier] full frame rows {err.max():.3e} columns {err2.max():.3e}", flush=True)
    assert err.max() <= 1e-5 and err2.max() <= 1e-5
