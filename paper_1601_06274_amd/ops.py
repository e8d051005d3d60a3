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

__all__ = ["DiscreteResult", "solve_discrete", "discrete_params", "tile_for"]


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
                    warm_start=False, tile=None) -> L.DmDiscreteParams:
    p = L.DmDiscreteParams()
    p.n_iters = int(n_iters)
    p.n_half_steps = int(n_half_steps)
    p.trunc_T = int(T)
    p.minorant = {"iterative": L.DM_MINORANT_ITERATIVE, "naive": L.DM_MINORANT_NAIVE}[minorant]
    gammas = tuple(gammas)
    p.max_pass = len(gammas)
    for i, g in enumerate(gammas[:8]):
        p.gamma[i] = float(g)
    p.warm_start = 1 if warm_start else 0
    if tile is not None:
        p.tile_lanes, p.labels_per_lane = int(tile[0]), int(tile[1])
    return p


@dataclass
class DiscreteResult:
    labels: torch.Tensor            # [H][W] int32
    minmarg: torch.Tensor | None    # [H][W][K] float32
    dual: torch.Tensor              # [H][W][K] float32
    bounds: torch.Tensor | None     # [2] float64: LB, E(labels)
    lb_trace: torch.Tensor | None   # [half-steps] float64


def tile_for(K: int):
    """Default (lanes per chain, labels per lane) the library picks for K labels."""
    tiles = [(4, 1), (4, 2), (8, 4), (16, 4), (32, 3), (32, 4), (64, 3), (64, 4)]
    best, waste = None, None
    for g, l in tiles:
        if g * l < K:
            continue
        w = g * l - K
        if best is None or w < waste or (w == waste and g > best[0]):
            best, waste = (g, l), w
    return best


def solve_discrete(cost, w_h, w_v, *, T=3, n_iters=10, n_half_steps=0, minorant="iterative",
                   gammas=(0.25, 0.25, 1.0), dual=None, warm_start=False, want_minmarg=True,
                   want_bounds=True, want_trace=False, tile=None, stream=None, workspace=None,
                   labels=None, minmarg=None) -> DiscreteResult:
    """Dual_MM on the GPU (dm_solve_discrete)."""
    H, W, K = cost.shape
    dev = cost.device
    _check_dev("cost", cost)
    _check_dev("w_h", w_h, torch.float32, (H, W - 1))
    _check_dev("w_v", w_v, torch.float32, (H - 1, W))
    dt = _cost_dtype(cost)
    p = discrete_params(T, n_iters, n_half_steps, minorant, gammas, warm_start, tile)
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
                          lb_trace=None if trace is None else trace[:S])
