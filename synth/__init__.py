"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module draws random numbers and builds images; it contains none of the
matching method's arithmetic (no cost volume, no message passing, no
refinement).  Every generator uses numpy's PCG64 so that one seed gives the
same arrays on every machine, and everything returned is a plain numpy array
that both the FP64 oracle and the GPU library consume unchanged.

Workload shapes follow the paper's experiments: 640x480 frames with 128
disparities (the live-camera setting of Sec. 4.1.2) and 1242x375 frames with
192 disparities (a driving-scene frame size).  Real images are replaced by a
generator with the same structure: textured left image, piecewise-planar
(slanted) disparity, occlusion bands and sensor noise.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "rng",
    "uniform_unaries",
    "tiny_instance",
    "StereoPair",
    "stereo_pair",
    "BatchSpec",
    "batch_specs",
    "FlowPair",
    "flow_pair",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for ``seed`` (the only RNG used by every input)."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_unaries(H: int, W: int, K: int, seed: int = 0, w: float = 0.1):
    """Unary volume theta[H][W][K] ~ U[0,1) (float32) and constant edge weights.

    Returns ``(theta, w_h, w_v)`` with ``w_h`` of shape (H, W-1) and ``w_v`` of
    shape (H-1, W), both filled with ``w`` (float32).
    """
    g = rng(seed)
    theta = g.random((H, W, K), dtype=np.float64).astype(np.float32)
    w_h = np.full((H, max(W - 1, 0)), w, dtype=np.float32)
    w_v = np.full((max(H - 1, 0), W), w, dtype=np.float32)
    return theta, w_h, w_v


def tiny_instance(H: int, W: int, K: int, seed: int, w_max: float = 0.6):
    """Small random instance: theta ~ U[0,1), per-edge weights ~ U[0, w_max)."""
    g = rng(seed)
    theta = g.random((H, W, K)).astype(np.float32)
    w_h = (g.random((H, max(W - 1, 0))) * w_max).astype(np.float32)
    w_v = (g.random((max(H - 1, 0), W)) * w_max).astype(np.float32)
    return theta, w_h, w_v


@dataclasses.dataclass
class StereoPair:
    left: np.ndarray       # [H][W] float32 in [0,1]
    right: np.ndarray      # [H][W] float32 in [0,1]
    disparity: np.ndarray  # [H][W] float32, true disparity in right-image coordinates
    K: int


def _box3(img: np.ndarray) -> np.ndarray:
    p = np.pad(img, 1, mode="edge")
    H, W = img.shape
    acc = np.zeros_like(img)
    for dy in range(3):
        for dx in range(3):
            acc += p[dy:dy + H, dx:dx + W]
    return acc / 9.0


def stereo_pair(W: int, H: int, K: int, seed: int, *, segments: int | None = None,
                slope: float = 0.02, occlusion_bands: int = 0,
                noise_sigma: float = 2.0 / 255.0) -> StereoPair:
    """Random-texture rectified stereo pair with piecewise-planar disparity.

    * left image: U[0,1) noise, 3x3 box blur, rescaled to [0,1];
    * disparity: Voronoi partition into ``segments`` cells, each a plane
      d = d0 + a (x - cx) + b (y - cy) with d0 ~ U[0.1K, 0.8K] and
      |a|, |b| <= ``slope``, clipped to [0, K-1];
    * right image: I_R(x', y) = I_L(x' + d(x', y), y) by linear interpolation;
    * ``occlusion_bands`` vertical bands (20-40 px wide) of I_R are replaced
      by fresh noise; then Gaussian noise of std ``noise_sigma`` is added and
      the result clipped to [0,1].
    """
    g = rng(seed)
    if segments is None:
        segments = max(4, int(round(W * H / 20000.0)))
    left = _box3(g.random((H, W)))
    lo, hi = left.min(), left.max()
    left = (left - lo) / max(hi - lo, 1e-12)

    cx = g.random(segments) * W
    cy = g.random(segments) * H
    d0 = g.uniform(0.1 * K, 0.8 * K, segments)
    a = g.uniform(-slope, slope, segments)
    b = g.uniform(-slope, slope, segments)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    best = np.full((H, W), np.inf)
    seg = np.zeros((H, W), dtype=np.int64)
    for s in range(segments):
        dist = (xs - cx[s]) ** 2 + (ys - cy[s]) ** 2
        closer = dist < best
        best[closer] = dist[closer]
        seg[closer] = s
    disp = d0[seg] + a[seg] * (xs - cx[seg]) + b[seg] * (ys - cy[seg])
    disp = np.clip(disp, 0.0, K - 1.0)

    src = np.clip(xs + disp, 0.0, W - 1.0)
    x0 = np.floor(src).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    t = src - x0
    rows = np.arange(H)[:, None]
    right = (1.0 - t) * left[rows, x0] + t * left[rows, x1]

    for _ in range(occlusion_bands):
        width = int(g.integers(20, 41))
        x_start = int(g.integers(0, max(W - width, 1)))
        right[:, x_start:x_start + width] = g.random((H, min(width, W - x_start)))

    right = right + g.normal(0.0, noise_sigma, right.shape)
    return StereoPair(
        left=left.astype(np.float32),
        right=np.clip(right, 0.0, 1.0).astype(np.float32),
        disparity=disp.astype(np.float32),
        K=K,
    )


@dataclasses.dataclass
class BatchSpec:
    W: int
    H: int
    K: int
    seed: int


def batch_specs(n: int = 64, seed: int = 4000, *, w_range=(160, 1280), h_range=(120, 720),
                k_choices=(32, 64, 128, 192)) -> list[BatchSpec]:
    """Uneven instance sizes: W ~ U{w_range}, H ~ U{h_range}, K from ``k_choices``."""
    g = rng(seed)
    out = []
    for i in range(n):
        W = int(g.integers(w_range[0], w_range[1] + 1))
        H = int(g.integers(h_range[0], h_range[1] + 1))
        K = int(k_choices[int(g.integers(0, len(k_choices)))])
        out.append(BatchSpec(W=W, H=H, K=K, seed=seed + 1 + i))
    return out


@dataclasses.dataclass
class FlowPair:
    first: np.ndarray   # [H][W] float32 in [0,1]
    second: np.ndarray  # [H][W] float32 in [0,1]
    flow: np.ndarray    # [H][W][2] float32: true displacement (horizontal, vertical), second-image grid


def flow_pair(W: int, H: int, max_disp: float, seed: int, *, segments: int | None = None, slope: float = 0.02,
              noise_sigma: float = 2.0 / 255.0) -> FlowPair:
    """Random-texture image pair related by a piecewise-affine flow.

    * first image: U[0,1) noise, 3x3 box blur, rescaled to [0,1];
    * flow: Voronoi partition into ``segments`` cells, each with an affine field
      u = u0 + A (p - c), u0 ~ U[-max_disp, max_disp]^2, |A_kl| <= ``slope``, clipped to
      [-max_disp, max_disp];
    * second image: I2(p) = I1(p - u(p)) by bilinear interpolation (clamped), plus Gaussian
      noise of std ``noise_sigma``, clipped to [0,1].
    """
    g = rng(seed)
    if segments is None:
        segments = max(3, int(round(W * H / 20000.0)))
    first = _box3(g.random((H, W)))
    lo, hi = first.min(), first.max()
    first = (first - lo) / max(hi - lo, 1e-12)
    cx = g.random(segments) * W
    cy = g.random(segments) * H
    u0 = g.uniform(-max_disp, max_disp, (segments, 2))
    A = g.uniform(-slope, slope, (segments, 2, 2))
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    best = np.full((H, W), np.inf)
    seg = np.zeros((H, W), dtype=np.int64)
    for s in range(segments):
        dist = (xs - cx[s]) ** 2 + (ys - cy[s]) ** 2
        closer = dist < best
        best[closer] = dist[closer]
        seg[closer] = s
    dx, dy = xs - cx[seg], ys - cy[seg]
    flow = np.stack([u0[seg, 0] + A[seg, 0, 0] * dx + A[seg, 0, 1] * dy,
                     u0[seg, 1] + A[seg, 1, 0] * dx + A[seg, 1, 1] * dy], axis=-1)
    flow = np.clip(flow, -max_disp, max_disp)
    sx = np.clip(xs - flow[..., 0], 0.0, W - 1.0)
    sy = np.clip(ys - flow[..., 1], 0.0, H - 1.0)
    x0 = np.floor(sx).astype(np.int64)
    y0 = np.floor(sy).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    t, s_ = sx - x0, sy - y0
    second = ((1 - s_) * ((1 - t) * first[y0, x0] + t * first[y0, x1])
              + s_ * ((1 - t) * first[y1, x0] + t * first[y1, x1]))
    second = second + g.normal(0.0, noise_sigma, second.shape)
    return FlowPair(first=first.astype(np.float32), second=np.clip(second, 0.0, 1.0).astype(np.float32),
                    flow=flow.astype(np.float32))
