"""Seeded synthetic workloads for the shiftable bilateral filter.

This module holds input generators only: it draws images and per-image filter
parameters from NumPy's PCG64 generator and holds none of the filter's
arithmetic.  The CPU oracle and the HIP path are both fed from here, so that
they see the same FP32 bytes.

The paper times its method on a 512x512 image it does not name (Section 2), and
uses no public benchmark or dataset, so the generators below are the whole
workload.  Axis convention: x is the column index, y the row index, 0-based;
images are row-major float32 arrays of shape (H, W).

Generators:
  smooth    128 + 60 sin(x/20) cos(y/15) + U(-40, 40), clipped to [0, 255]
  rect      background level U[0,255], then `n_rect` axis-aligned rectangles
            painted in order (later ones overwrite); each takes its corners
            from two sorted integer uniforms per axis over [0, W] and [0, H]
            and a level U[0,255]; then N(0, noise^2) is added and the result
            clipped to [0, 255]
  gradient  a linear ramp from level U[0,127] to U[128,255] along an angle
            U[0, 2 pi), the ramp spanning the image's extent along that
            direction, plus N(0, 20^2), clipped to [0, 255]
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "smooth_image",
    "rect_image",
    "gradient_image",
    "denoise_pair",
    "batch_specs",
    "random_image",
    "WORKLOADS",
]

LEVEL_MAX = 255.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


def smooth_image(H: int = 256, W: int = 256, seed: int = 1) -> np.ndarray:
    rng = _rng(seed)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    f = 128.0 + 60.0 * np.sin(x / 20.0) * np.cos(y / 15.0)
    f = f + rng.uniform(-40.0, 40.0, size=(H, W))
    return np.clip(f, 0.0, LEVEL_MAX).astype(np.float32)


def _paint_rects(rng: np.random.Generator, H: int, W: int, n_rect: int) -> np.ndarray:
    f = np.full((H, W), rng.uniform(0.0, LEVEL_MAX), dtype=np.float64)
    for _ in range(n_rect):
        x0, x1 = np.sort(rng.integers(0, W + 1, size=2))
        y0, y1 = np.sort(rng.integers(0, H + 1, size=2))
        level = rng.uniform(0.0, LEVEL_MAX)
        f[y0:y1, x0:x1] = level
    return f


def rect_image(H: int = 4096, W: int = 4096, seed: int = 2, n_rect: int = 64,
               noise: float = 20.0) -> np.ndarray:
    rng = _rng(seed)
    f = _paint_rects(rng, H, W, n_rect)
    if noise > 0:
        f = f + rng.normal(0.0, noise, size=(H, W))
    return np.clip(f, 0.0, LEVEL_MAX).astype(np.float32)


def gradient_image(H: int, W: int, seed: int, noise: float = 20.0) -> np.ndarray:
    rng = _rng(seed)
    lo = rng.uniform(0.0, 127.0)
    hi = rng.uniform(128.0, LEVEL_MAX)
    ang = rng.uniform(0.0, 2.0 * np.pi)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    p = x * np.cos(ang) + y * np.sin(ang)
    span = p.max() - p.min()
    t = (p - p.min()) / span if span > 0 else np.zeros_like(p)
    f = lo + (hi - lo) * t
    f = f + rng.normal(0.0, noise, size=(H, W))
    return np.clip(f, 0.0, LEVEL_MAX).astype(np.float32)


def denoise_pair(index: int, H: int = 1024, W: int = 1024, noise: float = 25.0):
    """(noisy input, clean target) for the differentiation workload.

    The target is a noise-free rect image; the input adds N(0, noise^2) and is
    clipped to [0, 255] so that every difference stays inside the range bound.
    Seed 5 + index.
    """
    rng = _rng(5 + index)
    target = np.clip(_paint_rects(rng, H, W, 64), 0.0, LEVEL_MAX)
    noisy = np.clip(target + rng.normal(0.0, noise, size=(H, W)), 0.0, LEVEL_MAX)
    return noisy.astype(np.float32), target.astype(np.float32)


def batch_specs(n: int = 256, seed: int = 4, side_lo: int = 128, side_hi: int = 2048,
                sigma_lo: float = 10.0, sigma_hi: float = 60.0, r_lo: int = 3, r_hi: int = 25):
    """Per-image (H, W, radius, sigma_r, image_seed) for the batched workload."""
    rng = _rng(seed)
    specs = []
    for i in range(n):
        H = int(rng.integers(side_lo, side_hi + 1))
        W = int(rng.integers(side_lo, side_hi + 1))
        sigma = float(rng.uniform(sigma_lo, sigma_hi))
        r = int(rng.integers(r_lo, r_hi + 1))
        specs.append((H, W, r, sigma, 1000 * seed + i))
    return specs


def random_image(H: int, W: int, seed: int, lo: float = 0.0, hi: float = LEVEL_MAX) -> np.ndarray:
    """Plain uniform noise, used by small parity and edge-case tests."""
    return _rng(seed).uniform(lo, hi, size=(H, W)).astype(np.float32)


# Named workloads: (generator, kwargs, radius, sigma_r, T, N or None for N_0).
WORKLOADS = {
    "smooth256_r5_s30": dict(gen="smooth", H=256, W=256, seed=1, radius=5, sigma_r=30.0, T=255.0, N=30),
    "rect4096_r20_s30": dict(gen="rect", H=4096, W=4096, seed=2, radius=20, sigma_r=30.0, T=255.0, N=30),
    "rect8192_r32_s15": dict(gen="rect", H=8192, W=8192, seed=3, radius=32, sigma_r=15.0, T=255.0, N=117),
    "denoise1024_r10_s25": dict(gen="denoise", H=1024, W=1024, seed=5, radius=10, sigma_r=25.0, T=255.0, N=43),
}


def make_image(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if w["gen"] == "smooth":
        return smooth_image(w["H"], w["W"], w["seed"])
    if w["gen"] == "rect":
        return rect_image(w["H"], w["W"], w["seed"])
    if w["gen"] == "denoise":
        return denoise_pair(0, w["H"], w["W"])[0]
    raise KeyError(name)
