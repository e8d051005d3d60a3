"""Python entry points with the C ABI's names (argument marshalling only).

Every step of the computation runs in the HIP library; torch supplies device
memory and the current stream.  Tensors must be CUDA (ROCm) tensors, contiguous,
in the layouts documented in include/dmatch.h.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

__all__ = ["DiscreteResult", "solve_discrete", "discrete_params", "tile_for", "refine_params", "refine_continuous",
           "build_cost_volume", "build_cost_volume_census", "lr_check", "build_flow_cost_volume", "flow_project",
           "refine_flow", "solve_flow", "FlowResult"]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(name, t, dtype=None, shape=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _cost_dtype(cost):
    if cost.dtype == torch.float32:
        return L.DM_F32
    if cost.dtype == torch.float16:
        return L.DM_F16
    raise ValueError("cost volume must be float32 or float16")


def discrete_params(T=3, n_iters=10, n_half_steps=0, minorant="iterative", gammas=(0.25, 0.25, 1.0),
                    warm_start=False, tile=None, keep_checkpoints=False,
                    recompute_selections=False) -> L.DmDiscreteParams:
    p = L.DmDiscreteParams()
    p.n_iters = int(n_iters)
    p.n_half_steps = int(n_half_steps)
    p.trunc_T = int(T)
    p.minorant = {"iterative": L.DM_MINORANT_ITERATIVE, "naive": L.DM_MINORANT_NAIVE,
                  "hierarchical": L.DM_MINORANT_HIERARCHICAL}[minorant]
    gammas = tuple(gammas)
    p.max_pass = len(gammas)
    for i, g in enumerate(gammas[:8]):
        p.gamma[i] = float(g)
    p.warm_start = 1 if warm_start else 0
    if tile is not None:
        # (lanes, labels per lane) for both families, or ((rows), (columns))
        if isinstance(tile[0], (tuple, list)):
            (p.tile_lanes, p.labels_per_lane), (p.tile_lanes_v, p.labels_per_lane_v) = tile
        else:
            p.tile_lanes, p.labels_per_lane = int(tile[0]), int(tile[1])
    # False/True -> 0/1 (dual checkpoints, messages recomputed); 2 or "record" -> 2 (the
    # forward also keeps every pass's messages and intermediate duals)
    p.keep_checkpoints = 2 if keep_checkpoints in (2, "record") else (1 if keep_checkpoints else 0)
    # the backward recomputes the selections instead of reading tapes (same results)
    p.recompute_selections = 1 if recompute_selections else 0
    return p


@dataclass
class DiscreteResult:
    labels: torch.Tensor            # [H][W] int32
    minmarg: torch.Tensor | None    # [H][W][K] float32
    dual: torch.Tensor              # [H][W][K] float32
    bounds: torch.Tensor | None     # [2] float64: LB, E(labels)
    lb_trace: torch.Tensor | None   # [half-steps] float64
    workspace: torch.Tensor | None = None  # holds the checkpoints when keep_checkpoints


def tile_for(K: int):
    """Default (lanes per chain, labels per lane) the library picks for K labels."""
    g, l = ctypes.c_int(0), ctypes.c_int(0)
    L.check("dm_default_tile", L.lib().dm_default_tile(int(K), ctypes.byref(g), ctypes.byref(l)))
    return g.value, l.value


def solve_discrete(cost, w_h, w_v, *, T=3, n_iters=10, n_half_steps=0, minorant="iterative",
                   gammas=(0.25, 0.25, 1.0), dual=None, warm_start=False, want_minmarg=True,
                   want_bounds=True, want_trace=False, tile=None, stream=None, workspace=None,
                   labels=None, minmarg=None, keep_checkpoints=False, recompute_selections=False) -> DiscreteResult:
    """Dual_MM on the GPU (dm_solve_discrete).  With keep_checkpoints the returned
    workspace holds what solve_discrete_backward needs (called with the same
    keep_checkpoints and recompute_selections)."""
    H, W, K = cost.shape
    dev = cost.device
    _check_dev("cost", cost)
    _check_dev("w_h", w_h, torch.float32, (H, W - 1))
    _check_dev("w_v", w_v, torch.float32, (H - 1, W))
    dt = _cost_dtype(cost)
    p = discrete_params(T, n_iters, n_half_steps, minorant, gammas, warm_start, tile, keep_checkpoints,
                        recompute_selections)
    shape = L.DmShape(W, H, K)
    lib = L.lib()
    ws_bytes = lib.dm_solve_discrete_workspace(shape, dt, ctypes.byref(p))
    if ws_bytes == 0:
        # the size query validates; call the solver to get the precise error
        ws_bytes = 256
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    if dual is None:
        dual = torch.empty((H, W, K), dtype=torch.float32, device=dev)
        if warm_start:
            raise ValueError("warm_start needs a dual tensor")
    _check_dev("dual", dual, torch.float32, (H, W, K))
    if labels is None:
        labels = torch.empty((H, W), dtype=torch.int32, device=dev)
    if want_minmarg and minmarg is None:
        minmarg = torch.empty((H, W, K), dtype=torch.float32, device=dev)
    if not want_minmarg:
        minmarg = None
    bounds = torch.empty(2, dtype=torch.float64, device=dev) if want_bounds else None
    S = n_half_steps if n_half_steps > 0 else 2 * n_iters
    trace = torch.empty(max(S, 1), dtype=torch.float64, device=dev) if want_trace else None
    st = lib.dm_solve_discrete(_ptr(cost), dt, _ptr(w_h), _ptr(w_v), shape, ctypes.byref(p), _ptr(labels),
                               _ptr(minmarg), _ptr(dual), _ptr(bounds), _ptr(trace), _ptr(workspace),
                               ctypes.c_size_t(workspace.numel()), _stream(stream))
    L.check("dm_solve_discrete", st)
    return DiscreteResult(labels=labels, minmarg=minmarg, dual=dual, bounds=bounds,
                          lb_trace=None if trace is None else trace[:S], workspace=workspace)


def solve_discrete_backward(cost, w_h, w_v, dual, fwd_workspace, *, grad_minmarg=None, grad_lb=0.0, grad_energy=0.0,
                            grad_bounds=None, T=3, n_iters=10, n_half_steps=0, minorant="iterative",
                            gammas=(0.25, 0.25, 1.0), tile=None, grad_cost=None, grad_w_h=None, grad_w_v=None,
                            accumulate=False, workspace=None, stream=None, keep_checkpoints=True,
                            recompute_selections=False):
    """Adjoint of solve_discrete (dm_solve_discrete_backward); the forward must have run with
    keep_checkpoints=True and the same parameters.  The bound gradients come either as a
    device float64 tensor ``grad_bounds`` = [dL/dLB, dL/dE] (read on the device) or as the
    numbers ``grad_lb`` and ``grad_energy``.  Returns (grad_cost, grad_w_h, grad_w_v)."""
    H, W, K = cost.shape
    dev = cost.device
    _check_dev("dual", dual, torch.float32, (H, W, K))
    _check_dev("grad_minmarg", grad_minmarg, torch.float32, (H, W, K))
    if grad_bounds is None and (float(grad_lb) != 0.0 or float(grad_energy) != 0.0):
        grad_bounds = torch.tensor([float(grad_lb), float(grad_energy)], dtype=torch.float64, device=dev)
    _check_dev("grad_bounds", grad_bounds, torch.float64, (2,))
    p = discrete_params(T, n_iters, n_half_steps, minorant, gammas, False, tile, keep_checkpoints or True,
                        recompute_selections)
    shape = L.DmShape(W, H, K)
    lib = L.lib()
    ws_bytes = max(int(lib.dm_solve_discrete_backward_workspace(shape, ctypes.byref(p))), 256)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    if grad_cost is None:
        grad_cost = torch.empty((H, W, K), dtype=torch.float32, device=dev)
    if grad_w_h is None:
        grad_w_h = torch.empty((H, W - 1), dtype=torch.float32, device=dev)
    if grad_w_v is None:
        grad_w_v = torch.empty((H - 1, W), dtype=torch.float32, device=dev)
    st = lib.dm_solve_discrete_backward(_ptr(grad_minmarg), _ptr(grad_bounds), _ptr(cost),
                                        _cost_dtype(cost), _ptr(w_h), _ptr(w_v), shape, ctypes.byref(p), _ptr(dual),
                                        _ptr(fwd_workspace), ctypes.c_size_t(fwd_workspace.numel()), _ptr(grad_cost),
                                        _ptr(grad_w_h), _ptr(grad_w_v), 1 if accumulate else 0, _ptr(workspace),
                                        ctypes.c_size_t(workspace.numel()), _stream(stream))
    L.check("dm_solve_discrete_backward", st)
    return grad_cost, grad_w_h, grad_w_v


def refine_params(C=3.0, eps=1.0, delta=0.0, h=1.0, tau=0.3, sigma=0.3, n_warps=5, n_iters=40,
                  keep_tape=False) -> L.DmRefineParams:
    return L.DmRefineParams(float(C), float(eps), float(delta), float(h), float(tau), float(sigma), int(n_warps),
                            int(n_iters), 1 if keep_tape else 0)


def refine_continuous(cost, labels, w_h, w_v, *, C=3.0, eps=1.0, delta=0.0, h=1.0, tau=0.3, sigma=0.3, n_warps=5,
                      n_iters=40, stream=None, workspace=None, u_out=None, keep_tape=False):
    """Warped non-linear primal-dual refinement (dm_refine_continuous); returns u [H][W] float32.
    With keep_tape the workspace (pass your own tensor) holds what the backward call needs."""
    H, W, K = cost.shape
    _check_dev("cost", cost)
    _check_dev("labels", labels, torch.int32, (H, W))
    _check_dev("w_h", w_h, torch.float32, (H, W - 1))
    _check_dev("w_v", w_v, torch.float32, (H - 1, W))
    p = refine_params(C, eps, delta, h, tau, sigma, n_warps, n_iters, keep_tape)
    shape = L.DmShape(W, H, K)
    lib = L.lib()
    ws_bytes = max(int(lib.dm_refine_continuous_workspace(shape, ctypes.byref(p))), 256)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=cost.device)
    if u_out is None:
        u_out = torch.empty((H, W), dtype=torch.float32, device=cost.device)
    st = lib.dm_refine_continuous(_ptr(cost), _cost_dtype(cost), _ptr(labels), _ptr(w_h), _ptr(w_v), shape,
                                  ctypes.byref(p), _ptr(u_out), _ptr(workspace), ctypes.c_size_t(workspace.numel()),
                                  _stream(stream))
    L.check("dm_refine_continuous", st)
    return u_out


def build_cost_volume(I_left, I_right, K, *, window=3, trunc=0.3, lambda_pw=0.1, contrast_sigma=0.1,
                      dtype=torch.float32, stream=None, cost_out=None, w_h=None, w_v=None):
    """Truncated windowed SAD cost volume and contrast weights (dm_build_cost_volume)."""
    H, W = I_left.shape
    _check_dev("I_left", I_left, torch.float32, (H, W))
    _check_dev("I_right", I_right, torch.float32, (H, W))
    dev = I_left.device
    if cost_out is None:
        cost_out = torch.empty((H, W, K), dtype=dtype, device=dev)
    if w_h is None:
        w_h = torch.empty((H, W - 1), dtype=torch.float32, device=dev)
    if w_v is None:
        w_v = torch.empty((H - 1, W), dtype=torch.float32, device=dev)
    cp = L.DmCostParams(int(window), float(trunc), float(lambda_pw), float(contrast_sigma))
    st = L.lib().dm_build_cost_volume(_ptr(I_left), _ptr(I_right), L.DmShape(W, H, K), ctypes.byref(cp),
                                      _cost_dtype(cost_out), _ptr(cost_out), _ptr(w_h), _ptr(w_v), _stream(stream))
    L.check("dm_build_cost_volume", st)
    return cost_out, w_h, w_v


def build_cost_volume_census(I_left, I_right, K, *, window=5, trunc=1.0, view="left", lambda_pw=0.1,
                             contrast_sigma=0.1, dtype=torch.float32, stream=None, cost_out=None, w_h=None,
                             w_v=None):
    """Census + Hamming cost volume of the left or right view and the view's contrast
    weights (dm_build_cost_volume_census)."""
    H, W = I_left.shape
    _check_dev("I_left", I_left, torch.float32, (H, W))
    _check_dev("I_right", I_right, torch.float32, (H, W))
    if view not in ("left", "right"):
        raise ValueError(f"view must be 'left' or 'right', got {view!r}")
    dev = I_left.device
    if cost_out is None:
        cost_out = torch.empty((H, W, K), dtype=dtype, device=dev)
    if w_h is None:
        w_h = torch.empty((H, W - 1), dtype=torch.float32, device=dev)
    if w_v is None:
        w_v = torch.empty((H - 1, W), dtype=torch.float32, device=dev)
    cp = L.DmCostParams(int(window), float(trunc), float(lambda_pw), float(contrast_sigma))
    st = L.lib().dm_build_cost_volume_census(_ptr(I_left), _ptr(I_right), L.DmShape(W, H, K), ctypes.byref(cp),
                                             0 if view == "left" else 1, _cost_dtype(cost_out), _ptr(cost_out),
                                             _ptr(w_h), _ptr(w_v), _stream(stream))
    L.check("dm_build_cost_volume_census", st)
    return cost_out, w_h, w_v


def lr_check(u_left, u_right, *, max_diff=1.0, invalid=-1.0, stream=None, out=None):
    """Left disparities kept where the right view agrees, `invalid` elsewhere (dm_lr_check)."""
    H, W = u_left.shape
    _check_dev("u_left", u_left, torch.float32, (H, W))
    _check_dev("u_right", u_right, torch.float32, (H, W))
    if out is None:
        out = torch.empty_like(u_left)
    _check_dev("out", out, torch.float32, (H, W))
    if out.data_ptr() in (u_left.data_ptr(), u_right.data_ptr()):
        raise ValueError("out must not alias u_left or u_right")
    st = L.lib().dm_lr_check(_ptr(u_left), _ptr(u_right), W, H, float(max_diff), float(invalid), _ptr(out),
                             _stream(stream))
    L.check("dm_lr_check", st)
    return out


def _flow_shape(H, W, K1, K2, off1, off2):
    return L.DmFlowShape(int(W), int(H), int(K1), int(K2), int(off1), int(off2))


def build_flow_cost_volume(I1, I2, K1, K2, off1, off2, *, window=3, trunc=0.3, lambda_pw=0.1, contrast_sigma=0.1,
                           dtype=torch.float32, stream=None, cost_out=None, w_h=None, w_v=None):
    """Two-dimensional truncated SAD flow cost [H][W][K2][K1] and the contrast weights of I1
    (dm_build_flow_cost_volume).  Label (i, j) is the displacement (i - off1, j - off2)."""
    H, W = I1.shape
    _check_dev("I1", I1, torch.float32, (H, W))
    _check_dev("I2", I2, torch.float32, (H, W))
    dev = I1.device
    if cost_out is None:
        cost_out = torch.empty((H, W, K2, K1), dtype=dtype, device=dev)
    _check_dev("cost_out", cost_out, None, (H, W, K2, K1))
    if w_h is None:
        w_h = torch.empty((H, W - 1), dtype=torch.float32, device=dev)
    if w_v is None:
        w_v = torch.empty((H - 1, W), dtype=torch.float32, device=dev)
    cp = L.DmCostParams(int(window), float(trunc), float(lambda_pw), float(contrast_sigma))
    st = L.lib().dm_build_flow_cost_volume(_ptr(I1), _ptr(I2), _flow_shape(H, W, K1, K2, off1, off2), ctypes.byref(cp),
                                           _cost_dtype(cost_out), _ptr(cost_out), _ptr(w_h), _ptr(w_v), _stream(stream))
    L.check("dm_build_flow_cost_volume", st)
    return cost_out, w_h, w_v


def flow_project(cost, *, stream=None, f1=None, f2=None):
    """Decoupled layer costs (dm_flow_project): f1 [H][W][K1] = min over the vertical label,
    f2 [H][W][K2] = min over the horizontal label, in the cost dtype."""
    H, W, K2, K1 = cost.shape
    _check_dev("cost", cost)
    if f1 is None:
        f1 = torch.empty((H, W, K1), dtype=cost.dtype, device=cost.device)
    if f2 is None:
        f2 = torch.empty((H, W, K2), dtype=cost.dtype, device=cost.device)
    _check_dev("f1", f1, cost.dtype, (H, W, K1))
    _check_dev("f2", f2, cost.dtype, (H, W, K2))
    st = L.lib().dm_flow_project(_ptr(cost), _cost_dtype(cost), _flow_shape(H, W, K1, K2, 0, 0), _ptr(f1), _ptr(f2),
                                 _stream(stream))
    L.check("dm_flow_project", st)
    return f1, f2


def refine_flow(cost, labels1, labels2, w_h, w_v, *, off1=0, off2=0, C=3.0, eps=1.0, delta=0.0, h=1.0, tau=0.3,
                sigma=0.3, n_warps=5, n_iters=40, stream=None, workspace=None, u1_out=None, u2_out=None):
    """Quadratic-fit refinement of both flow components (dm_refine_flow); returns (u1, u2)
    in label units."""
    H, W, K2, K1 = cost.shape
    _check_dev("cost", cost)
    _check_dev("labels1", labels1, torch.int32, (H, W))
    _check_dev("labels2", labels2, torch.int32, (H, W))
    _check_dev("w_h", w_h, torch.float32, (H, W - 1))
    _check_dev("w_v", w_v, torch.float32, (H - 1, W))
    p = refine_params(C, eps, delta, h, tau, sigma, n_warps, n_iters, False)
    shape = _flow_shape(H, W, K1, K2, off1, off2)
    lib = L.lib()
    ws_bytes = max(int(lib.dm_refine_flow_workspace(shape, ctypes.byref(p))), 256)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=cost.device)
    if u1_out is None:
        u1_out = torch.empty((H, W), dtype=torch.float32, device=cost.device)
    if u2_out is None:
        u2_out = torch.empty((H, W), dtype=torch.float32, device=cost.device)
    st = lib.dm_refine_flow(_ptr(cost), _cost_dtype(cost), _ptr(labels1), _ptr(labels2), _ptr(w_h), _ptr(w_v), shape,
                            ctypes.byref(p), _ptr(u1_out), _ptr(u2_out), _ptr(workspace),
                            ctypes.c_size_t(workspace.numel()), _stream(stream))
    L.check("dm_refine_flow", st)
    return u1_out, u2_out


@dataclass
class FlowResult:
    f1: torch.Tensor
    f2: torch.Tensor
    layer1: DiscreteResult
    layer2: DiscreteResult
    u1: torch.Tensor           # [H][W] horizontal component, label units (displacement u1 - off1)
    u2: torch.Tensor           # [H][W] vertical component, label units (displacement u2 - off2)


def solve_flow(cost, w_h, w_v, *, off1=0, off2=0, T=3, n_iters=20, refine=None, stream=None, two_streams=True,
               **discrete_kw):
    """The flow pipeline on a [H][W][K2][K1] cost: decoupled layer costs, one Dual_MM solve per
    layer, then the quadratic-fit refinement (dict of refine_flow parameters; None = the
    defaults, False = none).  Composes the C calls only.  The two layers are independent
    problems: with two_streams the second is solved on a forked stream (default priority),
    joined before the refinement (each layer's chains alone fill only part of the chip)."""
    f1, f2 = flow_project(cost, stream=stream)
    main = torch.cuda.current_stream(cost.device) if stream is None else stream
    r1 = solve_discrete(f1, w_h, w_v, T=T, n_iters=n_iters, stream=main, **discrete_kw)
    if two_streams:
        side = torch.cuda.Stream(device=cost.device)
        side.wait_stream(main)
        r2 = solve_discrete(f2, w_h, w_v, T=T, n_iters=n_iters, stream=side, **discrete_kw)
        # the allocator must not hand out what the side stream still uses
        for t in (f2, w_h, w_v, r2.labels, r2.minmarg, r2.dual, r2.bounds, r2.lb_trace, r2.workspace):
            if t is not None:
                t.record_stream(side)
        main.wait_stream(side)
    else:
        r2 = solve_discrete(f2, w_h, w_v, T=T, n_iters=n_iters, stream=main, **discrete_kw)
    if refine is False:
        u1, u2 = r1.labels.float(), r2.labels.float()
    else:
        u1, u2 = refine_flow(cost, r1.labels, r2.labels, w_h, w_v, off1=off1, off2=off2, stream=main,
                             **(refine or {}))
    return FlowResult(f1=f1, f2=f2, layer1=r1, layer2=r2, u1=u1, u2=u2)


def profiler_enable(kinds=None):
    """Record HIP-event timings of library launches of the given kinds (names of
    ``_lib.PROF_KINDS``; None = all).  Clears earlier records."""
    mask = 0xFFFF if kinds is None else sum(1 << L.PROF_KINDS[k] for k in kinds)
    L.check("dm_profiler_enable", L.lib().dm_profiler_enable(ctypes.c_uint(mask)))


def profiler_disable():
    L.check("dm_profiler_enable", L.lib().dm_profiler_enable(ctypes.c_uint(0)))


def profiler_query(kind: str):
    """(launches, total_ms, algorithmic_bytes) recorded for one kind."""
    n = ctypes.c_longlong(0)
    ms = ctypes.c_double(0.0)
    by = ctypes.c_double(0.0)
    L.check("dm_profiler_query", L.lib().dm_profiler_query(L.PROF_KINDS[kind], ctypes.byref(n), ctypes.byref(ms),
                                                          ctypes.byref(by)))
    return int(n.value), float(ms.value), float(by.value)


def refine_workspace_bytes(shape_hwk, keep_tape=False, **params):
    H, W, K = shape_hwk
    p = refine_params(keep_tape=keep_tape, **params)
    return int(L.lib().dm_refine_continuous_workspace(L.DmShape(W, H, K), ctypes.byref(p)))


def refine_continuous_backward(grad_u, cost, w_h, w_v, fwd_workspace, *, C=3.0, eps=1.0, delta=0.0, h=1.0, tau=0.3,
                               sigma=0.3, n_warps=5, n_iters=40, grad_cost=None, grad_w_h=None, grad_w_v=None,
                               accumulate=False, workspace=None, stream=None):
    """Adjoint of refine_continuous (dm_refine_continuous_backward).  ``fwd_workspace`` is the
    workspace tensor of a forward call made with keep_tape=True and the same parameters."""
    H, W, K = cost.shape
    _check_dev("grad_u", grad_u, torch.float32, (H, W))
    p = refine_params(C, eps, delta, h, tau, sigma, n_warps, n_iters, True)
    shape = L.DmShape(W, H, K)
    lib = L.lib()
    dev = cost.device
    ws_bytes = max(int(lib.dm_refine_continuous_backward_workspace(shape, ctypes.byref(p))), 256)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    if grad_cost is None:
        grad_cost = torch.empty((H, W, K), dtype=torch.float32, device=dev)
    if grad_w_h is None:
        grad_w_h = torch.empty((H, W - 1), dtype=torch.float32, device=dev)
    if grad_w_v is None:
        grad_w_v = torch.empty((H - 1, W), dtype=torch.float32, device=dev)
    st = lib.dm_refine_continuous_backward(_ptr(grad_u), _ptr(cost), _cost_dtype(cost), _ptr(w_h), _ptr(w_v), shape,
                                           ctypes.byref(p), _ptr(fwd_workspace), ctypes.c_size_t(fwd_workspace.numel()),
                                           _ptr(grad_cost), _ptr(grad_w_h), _ptr(grad_w_v), 1 if accumulate else 0,
                                           _ptr(workspace), ctypes.c_size_t(workspace.numel()), _stream(stream))
    L.check("dm_refine_continuous_backward", st)
    return grad_cost, grad_w_h, grad_w_v


def autotune_tiles(shape_hwk, cost_dtype=torch.float16, *, T=3, minorant="iterative", gammas=(0.25, 0.25, 1.0),
                   stream=None):
    """Fastest compiled tile for row and column chains of this shape (dm_autotune_tiles).
    Returns ((lanes, labels per lane) rows, (lanes, labels per lane) columns)."""
    H, W, K = shape_hwk
    p = discrete_params(T=T, n_iters=1, minorant=minorant, gammas=gammas)
    dt = L.DM_F16 if cost_dtype == torch.float16 else L.DM_F32
    st = L.lib().dm_autotune_tiles(L.DmShape(W, H, K), dt, ctypes.byref(p), _stream(stream))
    L.check("dm_autotune_tiles", st)
    return (p.tile_lanes, p.labels_per_lane), (p.tile_lanes_v, p.labels_per_lane_v)


class BatchedPlan:
    """Many uneven instances solved by one hipGraph launch (dm_plan_batched / dm_run_batched).

    ``instances``: list of dicts with GPU tensors ``cost`` [H][W][K] (all float32 or all
    float16), ``w_h``, ``w_v``; the plan allocates ``labels``, ``dual``, ``bounds``
    (float64 [LB, E(labels)], with want_bounds), ``minmarg`` (the final row pass's
    normalized min-marginals, with want_minmarg) and (with refinement) ``u`` for each
    instance unless given.  Keep the object alive while
    running; call ``close()`` (or drop it) to free the plan's device memory.
    """

    def __init__(self, instances, *, T=3, n_iters=20, n_half_steps=0, minorant="iterative",
                 gammas=(0.25, 0.25, 1.0), tile=None, refine=None, want_bounds=True, want_minmarg=False):
        self.instances = []
        arr = (L.DmInstance * len(instances))()
        dtype = instances[0]["cost"].dtype
        for i, inst in enumerate(instances):
            cost = inst["cost"]
            if cost.dtype != dtype:
                raise ValueError("all instances must share the cost dtype")
            H, W, K = cost.shape
            d = dict(inst)
            dev = cost.device
            d.setdefault("labels", torch.empty((H, W), dtype=torch.int32, device=dev))
            d.setdefault("dual", torch.empty((H, W, K), dtype=torch.float32, device=dev))
            if refine is not None:
                d.setdefault("u", torch.empty((H, W), dtype=torch.float32, device=dev))
            if want_bounds:
                d.setdefault("bounds", torch.empty(2, dtype=torch.float64, device=dev))
            if want_minmarg:
                d.setdefault("minmarg", torch.empty((H, W, K), dtype=torch.float32, device=dev))
            for k in ("cost", "w_h", "w_v", "labels", "dual"):
                _check_dev(k, d[k])
            _check_dev("bounds", d.get("bounds"), torch.float64, (2,))
            _check_dev("minmarg", d.get("minmarg"), torch.float32, (H, W, K))
            arr[i] = L.DmInstance(L.DmShape(W, H, K), _ptr(cost), _ptr(d["w_h"]), _ptr(d["w_v"]), _ptr(d["labels"]),
                                  _ptr(d["dual"]), _ptr(d.get("u")), _ptr(d.get("bounds")), _ptr(d.get("minmarg")))
            self.instances.append(d)
        p = discrete_params(T, n_iters, n_half_steps, minorant, gammas, False, tile, False)
        rp = None if refine is None else refine_params(**refine)
        handle = ctypes.c_void_p()
        self._lib = L.lib()
        st = self._lib.dm_plan_batched(arr, len(instances), _cost_dtype(instances[0]["cost"]), ctypes.byref(p),
                                       None if rp is None else ctypes.byref(rp), ctypes.byref(handle))
        L.check("dm_plan_batched", st)
        self.handle = handle

    @property
    def device_bytes(self):
        return int(self._lib.dm_plan_device_bytes(self.handle))

    def run(self, stream=None):
        L.check("dm_run_batched", self._lib.dm_run_batched(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.dm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedGradPlan:
    """Forward and backward of many instances as one hipGraph launch (dm_plan_batched_grad).

    ``instances``: list of dicts with GPU tensors ``cost`` [H][W][K] (all float32 or all
    float16), ``w_h``, ``w_v`` and the loss inputs ``grad_minmarg`` [H][W][K], ``grad_bounds``
    (float64 [2]), ``grad_u`` [H][W] (each optional).  The plan allocates, unless given,
    ``labels``, ``dual``, ``minmarg`` (when grad_minmarg is given), ``bounds``, ``u`` (with
    refinement) and the gradients ``grad_cost``, ``grad_w_h``, ``grad_w_v``; every run
    overwrites them.  With want_grad=False the plan is the forward only (no gradient
    buffers, no loss inputs).  The instances are spread over n_streams forked streams
    of the graph by size.
    """

    def __init__(self, instances, *, T=3, n_iters=20, n_half_steps=0, minorant="iterative",
                 gammas=(0.25, 0.25, 1.0), tile=None, keep_checkpoints=2, refine=None, n_streams=8,
                 want_grad=True):
        self.instances = []
        arr = (L.DmGradInstance * len(instances))()
        dtype = instances[0]["cost"].dtype
        for i, inst in enumerate(instances):
            cost = inst["cost"]
            if cost.dtype != dtype:
                raise ValueError("all instances must share the cost dtype")
            H, W, K = cost.shape
            d = dict(inst)
            dev = cost.device
            d.setdefault("labels", torch.empty((H, W), dtype=torch.int32, device=dev))
            d.setdefault("dual", torch.empty((H, W, K), dtype=torch.float32, device=dev))
            if d.get("grad_minmarg") is not None:
                d.setdefault("minmarg", torch.empty((H, W, K), dtype=torch.float32, device=dev))
            d.setdefault("bounds", torch.empty(2, dtype=torch.float64, device=dev))
            if refine is not None:
                d.setdefault("u", torch.empty((H, W), dtype=torch.float32, device=dev))
            if want_grad:
                d.setdefault("grad_cost", torch.empty((H, W, K), dtype=torch.float32, device=dev))
                d.setdefault("grad_w_h", torch.empty((H, W - 1), dtype=torch.float32, device=dev))
                d.setdefault("grad_w_v", torch.empty((H - 1, W), dtype=torch.float32, device=dev))
            else:
                keep_checkpoints = False
            _check_dev("cost", cost)
            for k, dt_, shp in (("w_h", torch.float32, (H, W - 1)), ("w_v", torch.float32, (H - 1, W)),
                                ("labels", torch.int32, (H, W)), ("dual", torch.float32, (H, W, K)),
                                ("minmarg", torch.float32, (H, W, K)), ("bounds", torch.float64, (2,)),
                                ("u", torch.float32, (H, W)), ("grad_minmarg", torch.float32, (H, W, K)),
                                ("grad_bounds", torch.float64, (2,)), ("grad_u", torch.float32, (H, W)),
                                ("grad_cost", torch.float32, (H, W, K)), ("grad_w_h", torch.float32, (H, W - 1)),
                                ("grad_w_v", torch.float32, (H - 1, W))):
                _check_dev(k, d.get(k), dt_, shp)
            arr[i] = L.DmGradInstance(L.DmShape(W, H, K), *[_ptr(d.get(k)) for k in (
                "cost", "w_h", "w_v", "labels", "dual", "minmarg", "bounds", "u", "grad_minmarg", "grad_bounds",
                "grad_u", "grad_cost", "grad_w_h", "grad_w_v")])
            self.instances.append(d)
        p = discrete_params(T, n_iters, n_half_steps, minorant, gammas, False, tile, keep_checkpoints)
        rp = None if refine is None else refine_params(keep_tape=True, **refine)
        handle = ctypes.c_void_p()
        self._lib = L.lib()
        st = self._lib.dm_plan_batched_grad(arr, len(instances), _cost_dtype(instances[0]["cost"]), ctypes.byref(p),
                                            None if rp is None else ctypes.byref(rp), int(n_streams),
                                            ctypes.byref(handle))
        L.check("dm_plan_batched_grad", st)
        self.handle = handle

    @property
    def device_bytes(self):
        return int(self._lib.dm_plan_device_bytes(self.handle))

    def run(self, stream=None):
        L.check("dm_run_batched", self._lib.dm_run_batched(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.dm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
