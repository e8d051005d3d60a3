#!/usr/bin/env python3
"""Benchmark: one frame of the discrete-continuous stereo hot path on one MI355X.

Workload (default): a 1242 x 375 stereo frame with K = 192 disparities from the
seeded synthetic generator (textured left image, slanted piecewise-planar
disparity, 4 occlusion bands, sensor noise; it stands in for driving-scene
frames of that size).  One step is

    build_cost_volume (3x3 SAD, truncated at 0.3, stored FP16; contrast weights)
    -> solve_discrete  (Dual_MM, 20 dual iterations, iterative minorant, T = 3)
    -> refine_continuous (5 warps x 40 primal-dual iterations)
    -> refine_continuous_backward -> solve_discrete_backward
       (dL/dcost and dL/dw for L = <G_m, min-marginals> + LB + <G_u, u>, seeded G)

on images already resident in HBM.  The forward keeps, per half-step, every pass's
selection tape (keep_checkpoints = 2; about 35 GB at this frame), so the backward
differentiates without recomputing; the same step with dual checkpoints only (the
backward recomputes every half-step) is timed beside it.  ``ms_per_step`` is forward
+ backward per frame; ``value`` is the forward's chain-DP label-node updates per frame
(every dual iteration visits every label-node in 8 chain sweeps, 4 per half-step, the
final labeling in 2 more) times frames per second of that step.  A forward-only loop
(dual checkpoints only) is timed first ("forward_only"; the plain sweeps' roofline
comes from it).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth

WORKLOAD = dict(W=1242, H=375, K=192, seed=3000, slope=0.08, occlusion_bands=4, segments=16,
                n_iters=20, T=3, gammas=(0.25, 0.25, 1.0), n_warps=5, refine_iters=40, C=3.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time of the oracle sample on all host workers")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (64 uneven instances) and differentiation (8 x 960x320x96) workloads")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for rocprofv3 counter runs: a known-size elementwise kernel, then 2 dual iterations "
                         "of the frame; prints the probe size")
    return ap.parse_args()


def _oracle_band(job):
    """One worker of the CPU baseline: the FP64 oracle, as it is, repeating horizontal
    half-steps on a band of rows and vertical half-steps on a band of columns of the
    frame for about target_s seconds.  Returns (label-node updates, seconds, reps)."""
    pair, wl, band, target_s = job
    from oracle import cost_volume as ocv, dmm as odmm
    rows, cols = 16, 32
    r0 = (band * rows) % (wl["H"] - rows + 1)
    c0 = (band * cols) % (wl["W"] - cols + 1)
    L_r, R_r = pair.left[r0:r0 + rows], pair.right[r0:r0 + rows]
    th_rows = ocv.sad_cost_volume(L_r, R_r, wl["K"])
    w_h, _ = ocv.contrast_weights(L_r)
    L_c, R_c = pair.left[:, c0:c0 + cols], pair.right[:, c0:c0 + cols]
    th_cols = ocv.sad_cost_volume(L_c, R_c, wl["K"])
    _, w_v = ocv.contrast_weights(L_c)
    updates = 0
    reps = 0
    t0 = time.perf_counter()
    while True:
        lam = np.zeros_like(th_rows)
        odmm.half_step(th_rows, lam, w_h, np.zeros((rows - 1, wl["W"])), wl["T"], "h", gammas=wl["gammas"])
        updates += th_rows.size * 4
        lam = np.zeros_like(th_cols)
        odmm.half_step(th_cols, lam, np.zeros((wl["H"], cols - 1)), w_v, wl["T"], "v", gammas=wl["gammas"])
        updates += th_cols.size * 4
        reps += 1
        if time.perf_counter() - t0 >= target_s:
            break
    return updates, time.perf_counter() - t0, reps


def host_workers():
    """Worker processes for the CPU baseline: the host's CPUs available to this process,
    at most 16 (the CPU share of one GPU on a shared multi-GPU host)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, min(n, 16))


def cpu_baseline(pair, wl, target_s):
    """The FP64 oracle, as it is, on a bounded sample of the same frame (horizontal
    half-steps on bands of 16 rows, vertical half-steps on bands of 32 columns), run by
    one process per host CPU (each on its own bands) and then by one process alone.
    Returns label-node updates / s (4 sweeps per half-step).  Runs before the GPU is
    initialised: the worker processes are forked copies of this one."""
    import multiprocessing as mp
    n = host_workers()
    with mp.get_context("fork").Pool(n) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_band, [(pair, wl, b, target_s) for b in range(n)])
        wall = time.perf_counter() - t0
    single_s = max(2.0, target_s / 2)
    u1, el1, reps1 = _oracle_band((pair, wl, 0, single_s))
    updates = sum(r[0] for r in res)
    reps = sum(r[2] for r in res)
    return {"value": updates / wall, "unit": "label-node updates/s", "cores": n, "kind": "oracle",
            "host_cpus": os.cpu_count(), "host_cpus_available": len(os.sched_getaffinity(0)),
            "cores_note": "one worker process per CPU available to this process, capped at 16: the CPU share "
                          "of one GPU on this host (the host's other CPUs serve its other GPUs)",
            "sample": f"{n} processes, each repeating (horizontal half-step on 16 rows x {wl['W']} + vertical "
                      f"half-step on 32 columns x {wl['H']}) of its own bands of the frame, K={wl['K']}, FP64 "
                      f"numpy, {reps} repetitions in {wall:.1f} s wall",
            "value_single_thread": u1 / el1,
            "sample_single_thread": f"one process, {reps1} repetitions on the first bands in {el1:.1f} s"}


def _timed(fn, reps, torch):
    """Mean milliseconds of fn() over reps runs (after one untimed run), stream-synchronised."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def batched_extra(torch, ops, dev, n=64, seed=4000, n_iters=20, T=3, warps=5, iters=40, reps=3):
    """64 uneven instances (W in [160, 1280], H in [120, 720], K in {32, 64, 128, 192}) of
    the stereo generator: the batched plan (FP16 cost, one hipGraph launch: Dual_MM 20
    iterations, labels and bounds of every instance, refinement 5 x 40) against the plain
    single-instance FP32 forward of the same work on the same GPU."""
    import synth
    specs = synth.batch_specs(n, seed=seed)
    inst16, inst32 = [], []
    for sp in specs:
        pair = synth.stereo_pair(sp.W, sp.H, sp.K, seed=sp.seed)
        IL = torch.from_numpy(pair.left).to(dev)
        IR = torch.from_numpy(pair.right).to(dev)
        c16, wh, wv = ops.build_cost_volume(IL, IR, sp.K, dtype=torch.float16)
        c32, _, _ = ops.build_cost_volume(IL, IR, sp.K, dtype=torch.float32)
        inst16.append(dict(cost=c16, w_h=wh, w_v=wv))
        inst32.append(dict(cost=c32, w_h=wh, w_v=wv))
    nodes = sum(sp.W * sp.H * sp.K for sp in specs)
    updates = nodes * (8 * n_iters + 2)
    rkw = dict(C=3.0, n_warps=warps, n_iters=iters)
    t0 = time.perf_counter()
    plan = ops.BatchedPlan(inst16, T=T, n_iters=n_iters, refine=rkw)
    plan_s = time.perf_counter() - t0
    try:
        ms_b = _timed(plan.run, reps, torch)
        dev_gb = plan.device_bytes / 1e9
        lb_le_e = bool(all(float(d["bounds"][0]) <= float(d["bounds"][1]) + 1e-6 * abs(float(d["bounds"][1]))
                           for d in plan.instances))
    finally:
        plan.close()
    # the same work as one graph of per-instance kernel chains on forked streams
    # (instances advance through their half-steps independently)
    splan = ops.BatchedGradPlan(inst16, T=T, n_iters=n_iters, refine=rkw, n_streams=8, want_grad=False)
    try:
        ms_s = _timed(splan.run, reps, torch)
    finally:
        splan.close()
    ws, rws = None, None
    duals = [torch.empty(d["cost"].shape, dtype=torch.float32, device=dev) for d in inst32]
    bounds = [torch.empty(2, dtype=torch.float64, device=dev) for _ in inst32]

    def plain():
        nonlocal ws, rws
        for d, lam, b in zip(inst32, duals, bounds):
            r = ops.solve_discrete(d["cost"], d["w_h"], d["w_v"], T=T, n_iters=n_iters, dual=lam, workspace=ws,
                                   want_bounds=True, want_minmarg=False)
            if ws is None or r.workspace.numel() > ws.numel():
                ws = r.workspace
            b.copy_(r.bounds)
            need = ops.refine_workspace_bytes(tuple(d["cost"].shape), **rkw)
            if rws is None or rws.numel() < need:
                rws = torch.empty(need, dtype=torch.uint8, device=dev)
            ops.refine_continuous(d["cost"], r.labels, d["w_h"], d["w_v"], workspace=rws, **rkw)
    ms_p = _timed(plain, reps, torch)
    return {"workload": f"{n} uneven stereo instances, W in [160,1280], H in [120,720], K in {{32,64,128,192}}, "
                        f"seed {seed}; Dual_MM {n_iters} its, T={T}, labels and bounds; refinement {warps}x{iters}",
            "bounds_lb_le_e_all": lb_le_e,
            "label_nodes": nodes, "plan_build_s": plan_s, "plan_device_GB": dev_gb,
            "batched_fp16_ms": ms_b, "batched_fp16_updates_per_s": updates / (ms_b * 1e-3),
            "streams_plan_fp16_ms": ms_s, "streams_plan_note": "per-instance kernel chains on 8 forked streams of "
                                                              "one graph (dm_plan_batched_grad, forward only)",
            "plain_fp32_ms": ms_p, "plain_fp32_updates_per_s": updates / (ms_p * 1e-3),
            "speedup_vs_plain_fp32": ms_p / ms_b}


def diff_extra(torch, ops, dev, n=8, W=960, H=320, K=96, n_iters=20, T=3, warps=1, iters=50, seed=5000, reps=2,
               n_streams=8):
    """Differentiation workload: a batch of 8 frames 960x320, K=96, FP16 cost; forward
    (Dual_MM 20 its keeping the selection tapes + refinement 1 x 50 steps) and backward
    (dL/dcost, dL/dw) of every frame as one batched plan (dm_plan_batched_grad: one
    hipGraph, frames on n_streams forked streams, each frame advancing on its own).
    Reported against the plain FP32 forward of the same frames (Dual_MM + refinement),
    one frame after another and on the same number of streams, and against the same
    forward + backward calls made eagerly one frame after another."""
    import ctypes
    import synth
    import paper_1601_06274_amd as P
    frames = []
    for i in range(n):
        pair = synth.stereo_pair(W, H, K, seed=seed + i, slope=0.08, occlusion_bands=2)
        IL = torch.from_numpy(pair.left).to(dev)
        IR = torch.from_numpy(pair.right).to(dev)
        c16, wh, wv = ops.build_cost_volume(IL, IR, K, dtype=torch.float16)
        c32, _, _ = ops.build_cost_volume(IL, IR, K, dtype=torch.float32)
        frames.append((c16, c32, wh, wv))
    dkw = dict(T=T, n_iters=n_iters)
    rkw = dict(C=3.0, n_warps=warps, n_iters=iters)
    gen = torch.Generator(device=dev).manual_seed(seed)
    G_m = torch.randn((H, W, K), generator=gen, device=dev)
    G_u = torch.randn((H, W), generator=gen, device=dev)
    G_b = torch.tensor([1.0, 0.0], dtype=torch.float64, device=dev)

    t0 = time.perf_counter()
    plan = ops.BatchedGradPlan([dict(cost=c16, w_h=wh, w_v=wv, grad_minmarg=G_m, grad_bounds=G_b, grad_u=G_u)
                                for c16, _, wh, wv in frames], keep_checkpoints=2, refine=rkw, n_streams=n_streams,
                               **dkw)
    plan_s = time.perf_counter() - t0
    try:
        ms_fb = _timed(plan.run, reps, torch)
        plan_gb = plan.device_bytes / 1e9
        # dL/dlambda_pw: the weights are lambda_pw * exp(...), so sum(dL/dw * w) / lambda_pw
        grad_lpw = [(d["grad_w_h"] * d["w_h"]).sum() + (d["grad_w_v"] * d["w_v"]).sum() for d in plan.instances]
        finite = bool(all(torch.isfinite(g).item() for g in grad_lpw) and
                      all(bool(torch.isfinite(d["grad_cost"]).all()) for d in plan.instances))
    finally:
        plan.close()

    # the same calls made eagerly, one frame after another on one stream
    lib = P.lib()
    shp = P._lib.DmShape(W, H, K)
    dp = ops.discrete_params(keep_checkpoints=2, **dkw)
    rp = ops.refine_params(keep_tape=True, **rkw)
    b = dict(ws_d=torch.empty(lib.dm_solve_discrete_workspace(shp, P._lib.DM_F16, ctypes.byref(dp)), dtype=torch.uint8,
                              device=dev),
             ws_db=torch.empty(lib.dm_solve_discrete_backward_workspace(shp, ctypes.byref(dp)), dtype=torch.uint8,
                               device=dev),
             ws_r=torch.empty(lib.dm_refine_continuous_workspace(shp, ctypes.byref(rp)), dtype=torch.uint8, device=dev),
             ws_rb=torch.empty(lib.dm_refine_continuous_backward_workspace(shp, ctypes.byref(rp)), dtype=torch.uint8,
                               device=dev),
             dual=torch.empty((H, W, K), dtype=torch.float32, device=dev),
             mm=torch.empty((H, W, K), dtype=torch.float32, device=dev),
             gc=torch.empty((H, W, K), dtype=torch.float32, device=dev),
             lab=torch.empty((H, W), dtype=torch.int32, device=dev), u=torch.empty((H, W), dtype=torch.float32,
                                                                                  device=dev),
             gwh=torch.empty((H, W - 1), dtype=torch.float32, device=dev),
             gwv=torch.empty((H - 1, W), dtype=torch.float32, device=dev))

    def eager_fwd_bwd():
        for c16, _, wh, wv in frames:
            ops.solve_discrete(c16, wh, wv, dual=b["dual"], workspace=b["ws_d"], labels=b["lab"], minmarg=b["mm"],
                               want_bounds=True, keep_checkpoints=2, **dkw)
            ops.refine_continuous(c16, b["lab"], wh, wv, workspace=b["ws_r"], u_out=b["u"], keep_tape=True, **rkw)
            ops.refine_continuous_backward(G_u, c16, wh, wv, b["ws_r"], grad_cost=b["gc"], grad_w_h=b["gwh"],
                                           grad_w_v=b["gwv"], accumulate=False, workspace=b["ws_rb"], **rkw)
            ops.solve_discrete_backward(c16, wh, wv, b["dual"], b["ws_d"], grad_minmarg=G_m, grad_bounds=G_b,
                                        grad_cost=b["gc"], grad_w_h=b["gwh"], grad_w_v=b["gwv"], accumulate=True,
                                        workspace=b["ws_db"], keep_checkpoints=2, **dkw)

    ms_fb_seq = _timed(eager_fwd_bwd, reps, torch)
    ckpt_gb = b["ws_d"].numel() / 1e9
    del b

    # the plain FP32 forward (no checkpoints), one frame after another and on n_streams streams
    fb = [dict(dual=torch.empty((H, W, K), dtype=torch.float32, device=dev),
               lab=torch.empty((H, W), dtype=torch.int32, device=dev),
               u=torch.empty((H, W), dtype=torch.float32, device=dev), ws32=None, ws_r=None)
          for _ in range(n_streams)]
    streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]

    def one_plain32(f, bb):
        _, c32, wh, wv = frames[f]
        r = ops.solve_discrete(c32, wh, wv, dual=bb["dual"], workspace=bb["ws32"], labels=bb["lab"],
                               want_bounds=False, want_minmarg=False, **dkw)
        bb["ws32"] = r.workspace
        if bb["ws_r"] is None:
            bb["ws_r"] = torch.empty(ops.refine_workspace_bytes((H, W, K), **rkw), dtype=torch.uint8, device=dev)
        ops.refine_continuous(c32, bb["lab"], wh, wv, u_out=bb["u"], workspace=bb["ws_r"], **rkw)

    def concurrent():
        main = torch.cuda.current_stream(dev)
        for st in streams:
            st.wait_stream(main)
        for f in range(n):
            k = f % n_streams
            with torch.cuda.stream(streams[k]):
                one_plain32(f, fb[k])
        for st in streams:
            main.wait_stream(st)

    def sequential():
        for f in range(n):
            one_plain32(f, fb[0])

    ms_32 = _timed(sequential, reps, torch)
    ms_32_conc = _timed(concurrent, reps, torch)
    return {"workload": f"batch of {n} frames {W}x{H}, K={K}, FP16 cost; Dual_MM {n_iters} its (tapes kept by the "
                        f"forward) + refinement {warps}x{iters}; backward dL/dcost, dL/dw (and dL/dlambda_pw); one "
                        f"batched plan (hipGraph, {n_streams} forked streams)",
            "fwd_bwd_fp16_ms_per_batch": ms_fb, "fwd_bwd_fp16_ms_per_frame": ms_fb / n,
            "fwd_bwd_fp16_eager_one_stream_ms_per_batch": ms_fb_seq,
            "plain_fp32_forward_ms_per_batch": ms_32, "plain_fp32_forward_streams_ms_per_batch": ms_32_conc,
            "ratio_fwd_bwd_to_plain_fwd": ms_fb / ms_32,
            "ratio_fwd_bwd_to_plain_fwd_same_streams": ms_fb / ms_32_conc,
            "plan_build_s": plan_s, "plan_device_GB": plan_gb,
            "checkpoint_GB_per_frame": ckpt_gb,
            "grad_finite": finite}


def _note(msg):
    """One progress line on stderr (the JSON result line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _traffic(traffic_file):
    """HBM bytes per launch from a stored rocprofv3 counter summary under profiles/, or None
    when there is none or the kernel's sources have changed since it was taken."""
    from paper_1601_06274_amd.traffic import source_hash
    tpath = os.path.join(ROOT, "profiles", traffic_file)
    if not os.path.exists(tpath):
        return None
    try:
        with open(tpath) as f:
            t = json.load(f)
        if t.get("kernel_source_hash") == source_hash(t.get("sources", "sweep")):
            return t.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


def hierarchical_extra(torch, ops, cost, w_h, w_v, wl, tiles, reps=2):
    """The hierarchical minorant (Handshake) against the iterative one on the bench frame's
    FP16 cost volume: Dual_MM forward time, per half-step kernel time and algorithmic
    GB/s, and the lower bound and labeling energy reached after 4 (the paper's live
    setting) and 20 dual iterations."""
    res = {}
    for mino in ("iterative", "hierarchical"):
        for its in (4, wl["n_iters"]):
            kw = dict(T=wl["T"], n_iters=its, minorant=mino, gammas=wl["gammas"], tile=tiles)
            r = ops.solve_discrete(cost, w_h, w_v, **kw)
            ws = r.workspace
            torch.cuda.synchronize()
            ops.profiler_enable(["sweep_h", "sweep_v"])
            ms = _timed(lambda: ops.solve_discrete(cost, w_h, w_v, workspace=ws, **kw), reps, torch)
            nh, msh, bh = ops.profiler_query("sweep_h")
            nv, msv, bv = ops.profiler_query("sweep_v")
            ops.profiler_disable()
            b = r.bounds.cpu().numpy()
            res[f"{mino}_{its}_its"] = {
                "forward_ms": ms, "lower_bound": float(b[0]), "energy": float(b[1]),
                "half_step_h_ms": msh / nh, "half_step_v_ms": msv / nv,
                "half_step_h_GBps": bh / (msh * 1e-3) / 1e9, "half_step_v_GBps": bv / (msv * 1e-3) / 1e9,
                "half_step_h_alg_bytes": bh / nh, "half_step_v_alg_bytes": bv / nv}
            if mino == "hierarchical":
                # HBM bytes per launch from rocprofv3 counters (null once the kernel source changed)
                res[f"{mino}_{its}_its"].update(half_step_h_traffic=_traffic("hier_h_traffic.json"),
                                                half_step_v_traffic=_traffic("hier_v_traffic.json"))
    return {"workload": f"{wl['W']}x{wl['H']}, K={wl['K']}, FP16 SAD cost, T={wl['T']}: Dual_MM with the iterative "
                        f"and the hierarchical minorant (labels, bounds, no refinement)", **res}


def flow_extra(torch, ops, dev, W=640, H=480, K=64, max_disp=24.0, seed=6000, n_iters=20, warps=5, iters=40,
               reps=3):
    """The optical-flow workload (Sec. 2.2 decoupled layer costs, Sec. 3.2 quadratic-fit
    refinement) on a synthetic 640x480 pair related by a piecewise-affine flow of up to
    24 px: the K x K two-dimensional SAD cost (FP16, displacements -32..31 on both axes),
    the two layer projections, one Dual_MM solve per layer (20 iterations) and the
    refinement of both components (5 x 40); per-stage times and the end-point error
    against the generator's flow.  The two layers' solves are timed one after the other
    and on two streams; total_ms takes the faster."""
    import synth
    pair = synth.flow_pair(W, H, max_disp, seed)
    I1 = torch.from_numpy(pair.first).to(dev)
    I2 = torch.from_numpy(pair.second).to(dev)
    off = K // 2
    cost, w_h, w_v = ops.build_flow_cost_volume(I1, I2, K, K, off, off, dtype=torch.float16)
    ms_cost = _timed(lambda: ops.build_flow_cost_volume(I1, I2, K, K, off, off, dtype=torch.float16, cost_out=cost,
                                                        w_h=w_h, w_v=w_v), reps, torch)
    f1, f2 = ops.flow_project(cost)
    ms_proj = _timed(lambda: ops.flow_project(cost, f1=f1, f2=f2), reps, torch)
    tiles = ops.autotune_tiles((H, W, K), torch.float16, T=3)
    kw = dict(T=3, n_iters=n_iters, tile=tiles)
    r1 = ops.solve_discrete(f1, w_h, w_v, **kw)
    r2 = ops.solve_discrete(f2, w_h, w_v, **kw)

    # every output and the duals preallocated: nothing is allocated per call, so the
    # second layer may run on another stream without the allocator recycling its memory
    out1 = dict(workspace=r1.workspace, labels=r1.labels, minmarg=r1.minmarg, dual=r1.dual, want_bounds=False)
    out2 = dict(workspace=r2.workspace, labels=r2.labels, minmarg=r2.minmarg, dual=r2.dual, want_bounds=False)

    def discrete():
        ops.solve_discrete(f1, w_h, w_v, **out1, **kw)
        ops.solve_discrete(f2, w_h, w_v, **out2, **kw)

    ms_dmm = _timed(discrete, reps, torch)
    # the two layers are independent problems: the second on a forked stream (default
    # priority), joined before the refinement
    s_a, s_b = torch.cuda.current_stream(), torch.cuda.Stream(device=dev)

    def discrete_two_streams():
        s_b.wait_stream(s_a)
        ops.solve_discrete(f1, w_h, w_v, stream=s_a, **out1, **kw)
        ops.solve_discrete(f2, w_h, w_v, stream=s_b, **out2, **kw)
        s_a.wait_stream(s_b)

    ms_dmm2 = _timed(discrete_two_streams, reps, torch)
    rkw = dict(off1=off, off2=off, C=3.0, n_warps=warps, n_iters=iters)
    ms_ref = _timed(lambda: ops.refine_flow(cost, r1.labels, r2.labels, w_h, w_v, **rkw), reps, torch)
    u1, u2 = ops.refine_flow(cost, r1.labels, r2.labels, w_h, w_v, **rkw)
    torch.cuda.synchronize()
    est = np.stack([u1.cpu().numpy() - off, u2.cpu().numpy() - off], axis=-1)
    disc = np.stack([r1.labels.cpu().numpy() - off, r2.labels.cpu().numpy() - off], axis=-1).astype(np.float64)
    epe = np.linalg.norm(est - pair.flow, axis=-1)
    epe_disc = np.linalg.norm(disc - pair.flow, axis=-1)
    updates = 2.0 * n_iters * 2 * W * H * K  # both layers, a row and a column half-step per iteration
    total = ms_cost + ms_proj + min(ms_dmm, ms_dmm2) + ms_ref
    return {"workload": f"optical flow {W}x{H}, {K}x{K} displacement labels (-{off}..{K - off - 1} px), FP16 2-D SAD "
                        f"cost, synthetic piecewise-affine flow up to {max_disp:g} px (seed {seed}); decoupled layer "
                        f"costs, Dual_MM {n_iters} its per layer, quadratic-fit refinement {warps}x{iters}",
            "cost_volume_ms": ms_cost, "cost_volume_GB": cost.numel() * 2 / 1e9, "projection_ms": ms_proj,
            "dual_mm_both_layers_ms": ms_dmm, "dual_mm_label_node_updates_per_s": updates / (ms_dmm * 1e-3),
            "dual_mm_layers_on_two_streams_ms": ms_dmm2,
            "refinement_ms": ms_ref, "total_ms": total,
            "epe_median_px": float(np.median(epe)), "epe_mean_px": float(epe.mean()),
            "epe_discrete_median_px": float(np.median(epe_disc))}


def census_lr_extra(torch, ops, dev, pair, wl, tiles, reps=3):
    """The paper's data term and its two-sided check on the bench frame: the Census
    (5 x 5) + Hamming cost volume, FP16, of the left and the right view, then one forward
    (Dual_MM 20 iterations + refinement) per view and the left-right check of the two
    refined disparity maps, against the left view alone."""
    W, H, K = wl["W"], wl["H"], wl["K"]
    IL = torch.from_numpy(pair.left).to(dev)
    IR = torch.from_numpy(pair.right).to(dev)
    views = {}
    for v in ("left", "right"):
        c, wh, wv = ops.build_cost_volume_census(IL, IR, K, window=5, view=v, dtype=torch.float16)
        views[v] = dict(cost=c, w_h=wh, w_v=wv, dual=torch.empty((H, W, K), dtype=torch.float32, device=dev),
                        labels=torch.empty((H, W), dtype=torch.int32, device=dev), ws=None, rws=None,
                        u=torch.empty((H, W), dtype=torch.float32, device=dev))
    ops.profiler_enable(["census", "lr_check"])
    for _ in range(reps):
        for v in ("left", "right"):
            ops.build_cost_volume_census(IL, IR, K, window=5, view=v, cost_out=views[v]["cost"],
                                         w_h=views[v]["w_h"], w_v=views[v]["w_v"])
    torch.cuda.synchronize()
    n_c, ms_c, by_c = ops.profiler_query("census")
    out_u = torch.empty((H, W), dtype=torch.float32, device=dev)

    # every buffer of a view preallocated (after the first, untimed call): nothing is
    # allocated per call, so the right view may run on another stream
    def forward(v, stream=None):
        d = views[v]
        r = ops.solve_discrete(d["cost"], d["w_h"], d["w_v"], T=wl["T"], n_iters=wl["n_iters"],
                               gammas=wl["gammas"], dual=d["dual"], labels=d["labels"], workspace=d["ws"],
                               want_minmarg=False, want_bounds=False, tile=tiles, stream=stream)
        d["ws"] = r.workspace
        if d["rws"] is None:
            d["rws"] = torch.empty(ops.refine_workspace_bytes((H, W, K), C=wl["C"], n_warps=wl["n_warps"],
                                                              n_iters=wl["refine_iters"]),
                                   dtype=torch.uint8, device=dev)
        ops.refine_continuous(d["cost"], r.labels, d["w_h"], d["w_v"], C=wl["C"], n_warps=wl["n_warps"],
                              n_iters=wl["refine_iters"], workspace=d["rws"], u_out=d["u"], stream=stream)

    def left_only():
        ops.build_cost_volume_census(IL, IR, K, window=5, view="left", cost_out=views["left"]["cost"],
                                     w_h=views["left"]["w_h"], w_v=views["left"]["w_v"])
        forward("left")

    def both():
        for v in ("left", "right"):
            ops.build_cost_volume_census(IL, IR, K, window=5, view=v, cost_out=views[v]["cost"],
                                         w_h=views[v]["w_h"], w_v=views[v]["w_v"])
            forward(v)
        ops.lr_check(views["left"]["u"], views["right"]["u"], max_diff=1.0, invalid=-1.0, out=out_u)

    # the two views are independent until the check: the right one on a forked stream
    # (default priority), joined before the check
    s_a, s_b = torch.cuda.current_stream(), torch.cuda.Stream(device=dev)

    def both_two_streams():
        s_b.wait_stream(s_a)
        for v, st in (("left", s_a), ("right", s_b)):
            ops.build_cost_volume_census(IL, IR, K, window=5, view=v, cost_out=views[v]["cost"],
                                         w_h=views[v]["w_h"], w_v=views[v]["w_v"], stream=st)
            forward(v, st)
        s_a.wait_stream(s_b)
        ops.lr_check(views["left"]["u"], views["right"]["u"], max_diff=1.0, invalid=-1.0, out=out_u)

    ms_left = _timed(left_only, reps, torch)
    ms_both = _timed(both, reps, torch)
    kept1 = out_u.clone()
    ms_both2 = _timed(both_two_streams, reps, torch)
    same = bool(torch.equal(kept1, out_u))
    n_l, ms_l, _ = ops.profiler_query("lr_check")
    ops.profiler_disable()
    kept = float((out_u >= 0).float().mean().item())
    gbs = by_c / (ms_c * 1e-3) / 1e9
    return {"workload": f"{W}x{H}, K={K}: Census 5x5 + Hamming cost volume (FP16) of both views, Dual_MM "
                        f"{wl['n_iters']} its + refinement per view, left-right check (max_diff 1)",
            "census_ms_per_view": ms_c / n_c, "census_GBps": gbs, "census_hbm_frac": gbs / HBM_PEAK_GBS,
            "census_alg_bytes_per_view": by_c / n_c,
            "lr_check_ms": ms_l / max(n_l, 1),
            "forward_left_view_ms": ms_left, "forward_both_views_and_check_ms": ms_both,
            "ratio_both_to_left": ms_both / ms_left,
            "forward_both_views_two_streams_and_check_ms": ms_both2, "ratio_two_streams_to_left": ms_both2 / ms_left,
            "two_streams_result_equal": same, "kept_fraction": kept}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); there is no multi-GPU path.",
              file=sys.stderr)
        return 2
    import synth

    wl = WORKLOAD
    W, H, K = wl["W"], wl["H"], wl["K"]
    pair = synth.stereo_pair(W, H, K, seed=wl["seed"], segments=wl["segments"], slope=wl["slope"],
                             occlusion_bands=wl["occlusion_bands"])
    # the CPU baseline forks its worker processes, so it runs before anything touches the GPU
    cpu = None if args.no_cpu_baseline or args.traffic_probe else cpu_baseline(pair, wl, args.cpu_seconds)
    import torch
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        return 1
    import paper_1601_06274_amd as P
    from paper_1601_06274_amd import ops
    dev = torch.device("cuda:0")
    IL = torch.from_numpy(pair.left).to(dev)
    IR = torch.from_numpy(pair.right).to(dev)
    cost = torch.empty((H, W, K), dtype=torch.float16, device=dev)
    w_h = torch.empty((H, W - 1), dtype=torch.float32, device=dev)
    w_v = torch.empty((H - 1, W), dtype=torch.float32, device=dev)
    dual = torch.empty((H, W, K), dtype=torch.float32, device=dev)
    minmarg = torch.empty((H, W, K), dtype=torch.float32, device=dev)
    labels = torch.empty((H, W), dtype=torch.int32, device=dev)
    u = torch.empty((H, W), dtype=torch.float32, device=dev)
    import ctypes
    lib = P.lib()
    shp = P._lib.DmShape(W, H, K)
    # chain tiles for row and column chains picked once by the library's autotuner
    tiles = ops.autotune_tiles((H, W, K), torch.float16, T=wl["T"], gammas=wl["gammas"])
    dkw = dict(T=wl["T"], n_iters=wl["n_iters"], gammas=wl["gammas"], tile=tiles)
    rkw = dict(C=wl["C"], n_warps=wl["n_warps"], n_iters=wl["refine_iters"])
    dp = ops.discrete_params(keep_checkpoints=True, **dkw)
    ws_d = torch.empty(lib.dm_solve_discrete_workspace(shp, P._lib.DM_F16, ctypes.byref(dp)), dtype=torch.uint8,
                       device=dev)
    ws_db = torch.empty(lib.dm_solve_discrete_backward_workspace(shp, ctypes.byref(dp)), dtype=torch.uint8, device=dev)
    rp = ops.refine_params(keep_tape=True, **rkw)
    ws_r = torch.empty(lib.dm_refine_continuous_workspace(shp, ctypes.byref(rp)), dtype=torch.uint8, device=dev)
    ws_rb = torch.empty(lib.dm_refine_continuous_backward_workspace(shp, ctypes.byref(rp)), dtype=torch.uint8,
                        device=dev)
    # loss L = <G_m, normalized min-marginals> + g_lb * LB + <G_u, u>, fixed seeded G
    gen = torch.Generator(device=dev).manual_seed(wl["seed"] + 1)
    G_m = torch.randn((H, W, K), generator=gen, device=dev, dtype=torch.float32)
    G_u = torch.randn((H, W), generator=gen, device=dev, dtype=torch.float32)
    g_lb = 1.0
    grad_cost = torch.empty((H, W, K), dtype=torch.float32, device=dev)
    grad_wh = torch.empty((H, W - 1), dtype=torch.float32, device=dev)
    grad_wv = torch.empty((H - 1, W), dtype=torch.float32, device=dev)

    if args.traffic_probe:
        n = 1 << 28  # 1 GiB of FP32: the in-place multiply reads and writes it once
        buf = torch.ones(n, dtype=torch.float32, device=dev)
        for _ in range(3):
            buf.mul_(1.0)
        del buf
        ops.build_cost_volume(IL, IR, K, dtype=torch.float16, cost_out=cost, w_h=w_h, w_v=w_v)
        k2 = dict(dkw, n_iters=2)
        # plain sweeps (dual checkpoints only), then the tape-recording forward and its backward
        ops.solve_discrete(cost, w_h, w_v, dual=dual, workspace=ws_d, labels=labels, minmarg=minmarg,
                           keep_checkpoints=True, **k2)
        del ws_d, ws_db
        dp2 = ops.discrete_params(keep_checkpoints=2, **k2)
        ws_d2 = torch.empty(lib.dm_solve_discrete_workspace(shp, P._lib.DM_F16, ctypes.byref(dp2)),
                            dtype=torch.uint8, device=dev)
        ws_db2 = torch.empty(lib.dm_solve_discrete_backward_workspace(shp, ctypes.byref(dp2)), dtype=torch.uint8,
                             device=dev)
        ops.solve_discrete(cost, w_h, w_v, dual=dual, workspace=ws_d2, labels=labels, minmarg=minmarg,
                           keep_checkpoints=2, **k2)
        ops.solve_discrete_backward(cost, w_h, w_v, dual, ws_d2, grad_minmarg=G_m, grad_lb=g_lb, grad_cost=grad_cost,
                                    grad_w_h=grad_wh, grad_w_v=grad_wv, workspace=ws_db2, keep_checkpoints=2, **k2)
        del ws_d2, ws_db2
        # the hierarchical minorant's half-steps (2 dual iterations)
        ops.solve_discrete(cost, w_h, w_v, T=wl["T"], n_iters=2, minorant="hierarchical", gammas=wl["gammas"],
                           tile=tiles)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe_bytes": 4 * n}), flush=True)
        return 0

    # keep_checkpoints = 2: the forward records every pass's selection tape (about 35 GB at
    # this frame, sized for 288 GB of HBM), the backward differentiates without recomputing.
    dp2 = ops.discrete_params(keep_checkpoints=2, **dkw)
    ws_d2 = torch.empty(lib.dm_solve_discrete_workspace(shp, P._lib.DM_F16, ctypes.byref(dp2)), dtype=torch.uint8,
                        device=dev)
    ws_db2 = torch.empty(lib.dm_solve_discrete_backward_workspace(shp, ctypes.byref(dp2)), dtype=torch.uint8,
                         device=dev)

    def forward(keep=True, ws=ws_d):
        ops.build_cost_volume(IL, IR, K, dtype=torch.float16, cost_out=cost, w_h=w_h, w_v=w_v)
        res = ops.solve_discrete(cost, w_h, w_v, dual=dual, workspace=ws, labels=labels, minmarg=minmarg,
                                 want_bounds=True, keep_checkpoints=keep, **dkw)
        ops.refine_continuous(cost, labels, w_h, w_v, workspace=ws_r, u_out=u, keep_tape=True, **rkw)
        return res

    def backward(keep=True, ws=ws_d, wsb=ws_db):
        ops.refine_continuous_backward(G_u, cost, w_h, w_v, ws_r, grad_cost=grad_cost, grad_w_h=grad_wh,
                                       grad_w_v=grad_wv, accumulate=False, workspace=ws_rb, **rkw)
        ops.solve_discrete_backward(cost, w_h, w_v, dual, ws, grad_minmarg=G_m, grad_lb=g_lb, grad_cost=grad_cost,
                                    grad_w_h=grad_wh, grad_w_v=grad_wv, accumulate=True, workspace=wsb,
                                    keep_checkpoints=keep, **dkw)

    def step():
        res = forward(2, ws_d2)
        backward(2, ws_d2, ws_db2)
        return res

    def step_recompute():
        forward(True, ws_d)
        backward(True, ws_d, ws_db)

    for _ in range(args.warmup):
        step()
        step_recompute()
    torch.cuda.synchronize()

    # Forward-only frames (dual checkpoints only); the sweep kernels are bracketed by HIP
    # events on their stream.
    ops.profiler_enable(["sweep_h", "sweep_v", "sweep_final", "cost_volume"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = forward()
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ops.profiler_disable()
    _note(f"forward-only frames: {fwd_ms:.2f} ms")

    prof = {k: ops.profiler_query(k) for k in ["sweep_h", "sweep_v", "sweep_final", "cost_volume"]}

    # Timed steps: forward (recording the tapes) + backward of the whole frame; the
    # record-mode and adjoint sweeps are bracketed by HIP events on their stream.
    bwd_kinds = ["adjoint_h", "adjoint_v", "adjoint_final", "record_h", "record_v"]
    ops.profiler_enable(bwd_kinds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ops.profiler_disable()
    ms_per_step = el * 1e3 / args.steps
    _note(f"timed steps: {ms_per_step:.2f} ms per step")
    grad_finite = bool(torch.isfinite(grad_cost).all().item() and torch.isfinite(grad_wh).all().item())
    prof.update({k: ops.profiler_query(k) for k in bwd_kinds})
    record_gb = (ws_d2.numel() + ws_db2.numel()) / 1e9

    def roof(kind, traffic_file, kernel):
        """Roofline object of one kernel kind: algorithmic bytes per launch / mean launch time."""
        n, ms, by = prof[kind]
        achieved = (by / n) / (ms / n * 1e-3) / 1e9 if n else 0.0
        traffic = _traffic(traffic_file)  # HBM bytes per launch from counters of the same kernel source
        return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "alg_bytes_per_launch": by / n if n else None,
                "avg_launch_ms": ms / n if n else None, "launches": n}
    n_h, ms_h, by_h = prof["sweep_h"]
    per_launch_gb = by_h / n_h / 1e9 if n_h else 0.0
    # sweep kernel kinds of the timed step (the traffic file of each, its description)
    STEP_KERNELS = {
        "adjoint_h": ("adjoint_h_traffic.json",
                      "adjoint of the horizontal half-step (R0 + 3 update passes in reverse, from the tapes)"),
        "record_h": ("record_h_traffic.json",
                     "horizontal half-step recording the selection tapes (R0 + 3 update passes, FP16 cost)"),
        "adjoint_v": ("adjoint_v_traffic.json", "adjoint of the vertical half-step (from the tapes)"),
        "record_v": ("record_v_traffic.json", "vertical half-step recording the selection tapes"),
    }
    dominant = max(STEP_KERNELS, key=lambda k: prof[k][1])
    del ws_d2, ws_db2
    torch.cuda.empty_cache()

    # The same step keeping only the dual before every half-step (keep_checkpoints = 1):
    # the backward recomputes each half-step from its checkpoint, recording its tapes.
    ms_recompute = _timed(step_recompute, max(2, args.steps // 2), torch)
    recompute_gb = (ws_d.numel() + ws_db.numel()) / 1e9

    # FP16 storage: energy of this labeling on the unrounded (FP32) costs vs the FP32-path
    # labeling, FP64 sums (outside the timed region)
    cost32 = torch.empty((H, W, K), dtype=torch.float32, device=dev)
    ops.build_cost_volume(IL, IR, K, dtype=torch.float32, cost_out=cost32, w_h=w_h, w_v=w_v)
    res32 = ops.solve_discrete(cost32, w_h, w_v, **dkw)
    e16 = _grid_energy(cost32, w_h, w_v, labels, wl["T"])
    e32 = _grid_energy(cost32, w_h, w_v, res32.labels, wl["T"])
    del cost32, res32

    N = H * W * K
    updates = N * (8 * wl["n_iters"] + 2)  # forward label-node updates per frame
    bounds = res.bounds.cpu().numpy()

    out = {
        "metric": "chain-DP label-node updates/s + HBM GB/s; fwd+bwd ms/frame at 1242x375x192",
        "value": updates / (ms_per_step * 1e-3),  # forward updates per frame x frames/s of fwd+bwd
        "unit": "label-node updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "stereo 1242x375, K=192 disparities, FP16 cost volume (3x3 SAD), Dual_MM 20 dual its "
                        "(iterative minorant 1/4,1/4,1, T=3) + refinement 5 warps x 40 its; step = forward + "
                        "backward (dL/dcost, dL/dw for L = <G_m, min-marginals> + LB + <G_u, u>); value counts "
                        "the forward's label-node updates per frame",
            "W": W, "H": H, "K": K, "cost_storage": "f16", "state": "f32",
            "tiles": {"rows": list(tiles[0]), "columns": list(tiles[1])},
            "stages": ["build_cost_volume", "solve_discrete", "refine_continuous", "refine_continuous_backward",
                       "solve_discrete_backward"],
        },
        "fwd_bwd_ms_per_frame": ms_per_step,
        "workspace_GB": record_gb,
        "fwd_bwd_recompute": {"ms_per_frame": ms_recompute, "workspace_GB": recompute_gb,
                              "note": "dual checkpoints only (keep_checkpoints=1); the backward recomputes each "
                                      "half-step, recording its tapes"},
        "forward_only": {"ms_per_frame": fwd_ms, "label_node_updates_per_s": updates / (fwd_ms * 1e-3)},
        "grad_finite": grad_finite,
        # the step's dominant kernel (largest total time among the sweep kinds of the step)
        "roofline": roof(dominant, STEP_KERNELS[dominant][0], STEP_KERNELS[dominant][1]),
        "roofline_step_kernels": {k: roof(k, f, d) for k, (f, d) in STEP_KERNELS.items()},
        "roofline_forward_sweep": roof("sweep_h", "sweep_h_traffic.json",
                                       "horizontal half-step chain sweep (R0 + 3 update passes, FP16 cost)"),
        "stage_ms": {
            "cost_volume": prof["cost_volume"][1] / max(prof["cost_volume"][0], 1),
            "sweep_h_per_launch": ms_h / max(n_h, 1),
            "sweep_v_per_launch": prof["sweep_v"][1] / max(prof["sweep_v"][0], 1),
            "sweep_v_GBps": (prof["sweep_v"][2] / prof["sweep_v"][1] / 1e6) if prof["sweep_v"][1] else None,
            "final_per_launch": prof["sweep_final"][1] / max(prof["sweep_final"][0], 1),
            "adjoint_h_per_launch": prof["adjoint_h"][1] / max(prof["adjoint_h"][0], 1),
            "adjoint_v_per_launch": prof["adjoint_v"][1] / max(prof["adjoint_v"][0], 1),
            "record_h_per_launch": prof["record_h"][1] / max(prof["record_h"][0], 1),
            "record_v_per_launch": prof["record_v"][1] / max(prof["record_v"][0], 1),
        },
        "fp16_storage": {"energy_fp16_labels": e16, "energy_fp32_labels": e32, "rel_diff": (e16 - e32) / e32},
        "lower_bound": float(bounds[0]),
        "energy": float(bounds[1]),
        "alg_gb_per_sweep_h": per_launch_gb,
    }
    if not args.no_extras:
        del ws_r, ws_rb
        torch.cuda.empty_cache()
        _note("extra: batched workload")
        out["batched"] = batched_extra(torch, ops, dev)
        torch.cuda.empty_cache()
        _note("extra: differentiation workload")
        out["differentiation"] = diff_extra(torch, ops, dev)
        torch.cuda.empty_cache()
        _note("extra: Census cost and left-right check")
        out["census_left_right"] = census_lr_extra(torch, ops, dev, pair, wl, tiles)
        torch.cuda.empty_cache()
        _note("extra: hierarchical minorant")
        out["hierarchical_minorant"] = hierarchical_extra(torch, ops, cost, w_h, w_v, wl, tiles)
        torch.cuda.empty_cache()
        _note("extra: optical flow")
        out["optical_flow"] = flow_extra(torch, ops, dev)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


def _grid_energy(cost, w_h, w_v, labels, T):
    """E(x) = sum of unaries + truncated-linear pairwise terms, FP64 sums (torch on the GPU)."""
    import torch
    lab = labels.long()
    e = cost.gather(2, lab.unsqueeze(2)).double().sum()
    dh = (lab[:, 1:] - lab[:, :-1]).abs().clamp(max=T).double()
    dv = (lab[1:, :] - lab[:-1, :]).abs().clamp(max=T).double()
    return float((e + (w_h.double() * dh).sum() + (w_v.double() * dv).sum()).item())


if __name__ == "__main__":
    sys.exit(main())
