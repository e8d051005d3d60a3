"""GPU tests of the batched form (dm_plan_batched / dm_run_batched) and the autotuner.

Every instance of a batch must equal its single-instance solve bit for bit when both
use the same chain tiles (same arithmetic per chain), on every replay of the graph,
with eager work and synchronisations between replays; and the oracle within the
parity tolerances.
"""
import numpy as np
import pytest

import synth
from oracle import dmm as odmm, energy as oenergy, refine as oref
from tests.parity import MM_RTOL, check_labels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_06274_amd import ops
    return ops


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _instances(specs, dtype=torch.float32):
    out = []
    for (H, W, K, seed) in specs:
        theta, w_h, w_v = synth.tiny_instance(H, W, K, seed=seed, w_max=0.4)
        out.append(dict(cost=_dev(theta, dtype), w_h=_dev(w_h), w_v=_dev(w_v), theta=theta, wh=w_h, wv=w_v))
    return out


SPECS = [(7, 11, 8, 1), (12, 5, 32, 2), (3, 30, 20, 3), (16, 16, 64, 4), (9, 23, 8, 5), (1, 17, 5, 6), (13, 1, 4, 7)]


@pytest.mark.parametrize("dtype,half", [(torch.float32, 0), (torch.float16, 0), (torch.float16, 5)])
def test_batched_equals_single_instance_bitwise(dtype, half):
    """Labels, duals, min-marginals and the lower bound bit for bit (the same chain optima
    summed in the same order); the energy of the labels to FP64 rounding (partial sums in
    another order).  half = 5: the last half-step is a row one, so the column optima come from
    the plan's column optimum pass."""
    ops = _need()
    insts = _instances(SPECS, dtype)
    print(f"[case] batched {len(insts)} instances {dtype} half-steps {half}", flush=True)
    tiles = {}
    for d in insts:
        K = d["cost"].shape[2]
        tiles[K] = ops.tile_for(K)
    # one fixed tile per K: give the plan the per-K default through single-K batches
    plan = ops.BatchedPlan([{k: d[k] for k in ("cost", "w_h", "w_v")} for d in insts], T=3, n_iters=3,
                           n_half_steps=half, tile=None, want_minmarg=True)
    try:
        singles = []
        for d in insts:
            K = d["cost"].shape[2]
            tr, tc = ops.autotune_tiles(tuple(d["cost"].shape), dtype, T=3)
            singles.append(ops.solve_discrete(d["cost"], d["w_h"], d["w_v"], T=3, n_iters=3, n_half_steps=half,
                                              tile=(tr, tc)))
        torch.cuda.synchronize()
        for rep in range(3):
            plan.run()
            torch.cuda.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
            for i, (pi, s) in enumerate(zip(plan.instances, singles)):
                assert torch.equal(pi["labels"], s.labels), f"replay {rep} instance {i} labels"
                assert torch.equal(pi["dual"], s.dual), f"replay {rep} instance {i} dual"
                assert torch.equal(pi["minmarg"], s.minmarg), f"replay {rep} instance {i} min-marginals"
                b, bs = pi["bounds"].cpu().numpy(), s.bounds.cpu().numpy()
                assert b[0] == bs[0], f"replay {rep} instance {i} lower bound {b[0]} vs {bs[0]}"
                assert b[1] == pytest.approx(bs[1], rel=1e-12, abs=1e-12), f"replay {rep} instance {i} energy"
    finally:
        plan.close()


def test_batched_oracle_parity_and_refinement():
    ops = _need()
    specs = [(6, 9, 8, 11), (10, 7, 16, 12), (5, 14, 12, 13)]
    insts = _instances(specs)
    plan = ops.BatchedPlan([{k: d[k] for k in ("cost", "w_h", "w_v")} for d in insts], T=2, n_iters=2,
                           refine=dict(C=2.0, n_warps=2, n_iters=10))
    try:
        plan.run()
        torch.cuda.synchronize()
        for d, pi in zip(insts, plan.instances):
            th = d["theta"].astype(np.float64)
            ref = odmm.solve_discrete(th, d["wh"], d["wv"], 2, 2)
            lab = pi["labels"].cpu().numpy()
            ndiff, nbad = check_labels(lab, ref.labels, ref.minmarg, th)
            assert nbad == 0
            np.testing.assert_allclose(pi["dual"].cpu().numpy(), ref.lam, atol=1e-4)
            # bounds against the oracle's lower bound and the FP64 energy of the GPU labels
            b = pi["bounds"].cpu().numpy()
            scale = max(abs(ref.lower_bound), 1.0)
            assert abs(b[0] - ref.lower_bound) <= 1e-5 * scale
            assert b[1] == pytest.approx(oenergy.grid_energy(th, d["wh"], d["wv"], 2, lab), rel=1e-9, abs=1e-9)
            assert b[0] <= b[1] + 1e-6 * scale
            P32 = oref.RefineParams(C=2.0, tau=float(np.float32(0.3)), sigma=float(np.float32(0.3)), n_warps=2,
                                    n_iters=10)
            u_ref = oref.refine_continuous(th, d["wh"], d["wv"], lab, P32)
            assert np.abs(pi["u"].cpu().numpy() - u_ref).max() <= 1e-4
    finally:
        plan.close()


def test_batched_uneven_random_sizes():
    """A small draw of the uneven-size recipe (sizes scaled down): plan, two replays, checks."""
    ops = _need()
    specs = synth.batch_specs(6, seed=4000, w_range=(20, 90), h_range=(12, 50), k_choices=(8, 16, 32))
    insts = []
    for sp in specs:
        pair = synth.stereo_pair(sp.W, sp.H, sp.K, seed=sp.seed)
        from oracle import cost_volume as ocv
        th = ocv.sad_cost_volume(pair.left, pair.right, sp.K).astype(np.float16)
        wh, wv = ocv.contrast_weights(pair.left)
        insts.append(dict(cost=_dev(th, torch.float16), w_h=_dev(wh), w_v=_dev(wv), theta=th, wh=wh, wv=wv))
    plan = ops.BatchedPlan([{k: d[k] for k in ("cost", "w_h", "w_v")} for d in insts], T=3, n_iters=3)
    try:
        for _ in range(2):
            plan.run()
            torch.cuda.synchronize()
            for d, pi in zip(insts, plan.instances):
                ref = odmm.solve_discrete(d["theta"].astype(np.float64), d["wh"], d["wv"], 3, 3)
                lab = pi["labels"].cpu().numpy()
                _, nbad = check_labels(lab, ref.labels, ref.minmarg, d["theta"].astype(np.float64))
                assert nbad == 0
    finally:
        plan.close()


def test_autotuner_returns_valid_tiles():
    ops = _need()
    for shape in [(20, 40, 32), (30, 25, 192), (9, 9, 5)]:
        (gr, lr), (gc, lc) = ops.autotune_tiles(shape, torch.float16)
        assert gr * lr >= shape[2] and gc * lc >= shape[2]


def test_batched_full_64_instances_sampled():
    """The batched workload at its full size (64 uneven instances, W in [160, 1280], H in
    [120, 720], K in {32, 64, 128, 192} from seed 4000, FP16 cost, 20 dual iterations, one
    graph launch): the smallest and the largest instance of every K equal their
    single-instance solves with the plan's tiles (autotuned per K on the largest instance
    of that K) bit for bit.  The single-instance path is checked against the oracle at the
    full frame size in test_gpu_fullsize."""
    ops = _need()
    specs = synth.batch_specs(64, seed=4000)
    insts = []
    for sp in specs:
        pair = synth.stereo_pair(sp.W, sp.H, sp.K, seed=sp.seed)
        c16, wh, wv = ops.build_cost_volume(_dev(pair.left), _dev(pair.right), sp.K, dtype=torch.float16)
        insts.append(dict(cost=c16, w_h=wh, w_v=wv))
    print(f"[case] batched full: {len(insts)} instances, "
          f"{sum(sp.W * sp.H * sp.K for sp in specs) / 1e9:.2f} G label-nodes", flush=True)
    plan = ops.BatchedPlan(insts, T=3, n_iters=20)
    try:
        plan.run()
        torch.cuda.synchronize()
        by_k = {}
        for i, sp in enumerate(specs):
            by_k.setdefault(sp.K, []).append(i)
        checked = 0
        for K, idx in sorted(by_k.items()):
            area = lambda i: specs[i].W * specs[i].H
            big = max(idx, key=area)
            tiles = ops.autotune_tiles((specs[big].H, specs[big].W, K), torch.float16, T=3)
            for i in sorted({min(idx, key=area), big}):
                d = insts[i]
                s = ops.solve_discrete(d["cost"], d["w_h"], d["w_v"], T=3, n_iters=20, tile=tiles)
                torch.cuda.synchronize()
                assert torch.equal(plan.instances[i]["labels"], s.labels), f"instance {i} labels"
                assert torch.equal(plan.instances[i]["dual"], s.dual), f"instance {i} dual"
                checked += 1
        assert checked >= 4
    finally:
        plan.close()


def _eager_fwd_bwd(ops, d, kw, rkw):
    """One instance's forward and backward through the single-instance calls."""
    r = ops.solve_discrete(d["cost"], d["w_h"], d["w_v"], keep_checkpoints=2, **kw)
    rws = torch.empty(ops.refine_workspace_bytes(tuple(d["cost"].shape), keep_tape=True, **rkw), dtype=torch.uint8,
                      device="cuda")
    u = ops.refine_continuous(d["cost"], r.labels, d["w_h"], d["w_v"], keep_tape=True, workspace=rws, **rkw)
    gc, gwh, gwv = ops.refine_continuous_backward(d["grad_u"], d["cost"], d["w_h"], d["w_v"], rws, **rkw)
    ops.solve_discrete_backward(d["cost"], d["w_h"], d["w_v"], r.dual, r.workspace, grad_minmarg=d["grad_minmarg"],
                                grad_bounds=d["grad_bounds"], grad_cost=gc, grad_w_h=gwh, grad_w_v=gwv,
                                accumulate=True, keep_checkpoints=2, **kw)
    torch.cuda.synchronize()
    return dict(labels=r.labels, dual=r.dual, minmarg=r.minmarg, bounds=r.bounds, u=u, grad_cost=gc, grad_w_h=gwh,
                grad_w_v=gwv)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_batched_grad_plan_equals_eager(dtype):
    """dm_plan_batched_grad: uneven instances on 2 forked streams of one graph (two
    instances share a stream and its workspaces); every output and gradient equals the
    same single-instance calls made eagerly, bit for bit, on every replay."""
    ops = _need()
    specs = [(6, 9, 8, 21), (10, 7, 16, 22), (5, 14, 12, 23), (4, 6, 5, 24), (8, 8, 24, 25)]
    insts = _instances(specs, dtype)
    g = torch.Generator(device="cuda").manual_seed(7)
    for d in insts:
        H, W, K = d["cost"].shape
        d["grad_minmarg"] = torch.randn((H, W, K), generator=g, device="cuda")
        d["grad_u"] = torch.randn((H, W), generator=g, device="cuda")
        d["grad_bounds"] = torch.tensor([0.7, 0.3], dtype=torch.float64, device="cuda")
    kw = dict(T=3, n_iters=2)
    rkw = dict(C=3.0, n_warps=2, n_iters=9)
    keys = ("cost", "w_h", "w_v", "grad_minmarg", "grad_bounds", "grad_u")
    print(f"[case] batched grad plan {len(insts)} instances {dtype}", flush=True)
    plan = ops.BatchedGradPlan([{k: d[k] for k in keys} for d in insts], refine=rkw, n_streams=2, **kw)
    try:
        refs = [_eager_fwd_bwd(ops, d, kw, rkw) for d in insts]
        for rep in range(2):
            plan.run()
            torch.cuda.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
            for i, (pi, ref) in enumerate(zip(plan.instances, refs)):
                for k, v in ref.items():
                    assert torch.equal(pi[k], v), f"replay {rep} instance {i}: {k} differs"
    finally:
        plan.close()


@pytest.mark.parametrize("n_streams", [1, 3])
def test_batched_forward_plan_on_streams_equals_eager(n_streams):
    """dm_plan_batched_grad without gradients: each instance's Dual_MM and refinement on
    forked streams of one graph (instances spread by size); labels, duals, min-marginals,
    bounds and refined disparities equal the single-instance calls bit for bit."""
    ops = _need()
    specs = [(6, 9, 8, 31), (10, 7, 16, 32), (5, 14, 12, 33), (4, 6, 5, 34), (8, 8, 24, 35), (3, 11, 9, 36)]
    insts = _instances(specs, torch.float16)
    kw = dict(T=3, n_iters=3)
    rkw = dict(C=3.0, n_warps=2, n_iters=9)
    plan = ops.BatchedGradPlan([{k: d[k] for k in ("cost", "w_h", "w_v")} for d in insts], refine=rkw,
                               n_streams=n_streams, want_grad=False, **kw)
    try:
        refs = []
        for d in insts:
            r = ops.solve_discrete(d["cost"], d["w_h"], d["w_v"], want_minmarg=False, **kw)
            u = ops.refine_continuous(d["cost"], r.labels, d["w_h"], d["w_v"], **rkw)
            refs.append(dict(labels=r.labels, dual=r.dual, bounds=r.bounds, u=u))
        torch.cuda.synchronize()
        for rep in range(2):
            plan.run()
            torch.cuda.synchronize()
            for i, (pi, ref) in enumerate(zip(plan.instances, refs)):
                for k, v in ref.items():
                    assert torch.equal(pi[k], v), f"replay {rep} instance {i}: {k} differs"
    finally:
        plan.close()
