"""Seeded synthetic frames shaped like planar laser-induced fluorescence
(PLIF) droplet images: bright isotropic Gaussian spots on a dark, noisy
background.

This module serves both the oracle tests and the GPU tests and the benchmark.
It only draws random numbers and renders blob profiles; it holds none of the
detector's arithmetic.  The paper's own data (rendered spheres with Poisson and
Gaussian noise, 1000x1000, about 100-1000 blobs per frame; real PLIF frames)
is not available, so these frames stand in for it.

Workloads (all fp32, row-major):
  * ``small``  : one 256x256 frame, U[0, 0.05) noise + 20 blobs of amplitude 1,
                 std U[1, 8], centres uniform; ladder 1..8, ratio 1.6,
                 threshold 0.1, overlap 0.5.
  * ``frame1k``: one 1024x1024 frame of uint16 camera counts: Poisson noise
                 around a mean of 200 plus 500 blobs of std U[1, 30] and
                 amplitude U[0.25, 0.9] of full scale, clipped to 65535,
                 divided by 65535; ladder 1..30, ratio 1.6, threshold 0.05.
  * ``batch64``: 64 such 1024x1024 frames, blob count U{100..1000} each.
  * ``mixed128``: 128 frames of side S in {256, 512, 768, 1024, 1536, 2048},
                 square or a (S/2) x S crop with probability 1/2, one blob per
                 2000 px, content as ``frame1k``.
  * ``stream``: Poisson arrivals at 200 frames/s, sizes as ``mixed128``.
"""
from __future__ import annotations

import numpy as np

SIDES = (256, 512, 768, 1024, 1536, 2048)


def render_blobs(H: int, W: int, cy, cx, s, amp, out: np.ndarray | None = None) -> np.ndarray:
    """Add sum_b amp_b * exp(-((y-cy_b)^2 + (x-cx_b)^2) / (2 s_b^2)) to a
    float64 H x W canvas, each blob rendered inside +-7 s_b of its centre."""
    if out is None:
        out = np.zeros((H, W), np.float64)
    for y0, x0, sb, ab in zip(np.atleast_1d(cy), np.atleast_1d(cx), np.atleast_1d(s),
                              np.atleast_1d(amp)):
        h = 7.0 * sb
        ya, yb = max(0, int(np.floor(y0 - h))), min(H, int(np.ceil(y0 + h)) + 1)
        xa, xb = max(0, int(np.floor(x0 - h))), min(W, int(np.ceil(x0 + h)) + 1)
        if ya >= yb or xa >= xb:
            continue
        gy = np.exp(-((np.arange(ya, yb) - y0) ** 2) / (2.0 * sb * sb))
        gx = np.exp(-((np.arange(xa, xb) - x0) ** 2) / (2.0 * sb * sb))
        out[ya:yb, xa:xb] += ab * np.outer(gy, gx)
    return out


def small_frame(seed: int = 0, H: int = 256, W: int = 256, n_blobs: int = 20) -> np.ndarray:
    """Uniform [0, 0.05) noise plus n_blobs unit-amplitude blobs, std U[1, 8]."""
    rng = np.random.default_rng(seed)
    img = rng.uniform(0.0, 0.05, size=(H, W))
    cy = rng.uniform(0, H, n_blobs)
    cx = rng.uniform(0, W, n_blobs)
    s = rng.uniform(1.0, 8.0, n_blobs)
    render_blobs(H, W, cy, cx, s, np.ones(n_blobs), out=img)
    return img.astype(np.float32)


def camera_frame(seed: int, H: int = 1024, W: int = 1024, n_blobs: int = 500,
                 smin: float = 1.0, smax: float = 30.0, background: float = 200.0) -> np.ndarray:
    """uint16 camera counts (Poisson around background + blobs), returned as
    counts / 65535 in fp32."""
    rng = np.random.default_rng(seed)
    cy = rng.uniform(0, H, n_blobs)
    cx = rng.uniform(0, W, n_blobs)
    s = rng.uniform(smin, smax, n_blobs)
    amp = rng.uniform(0.25, 0.9, n_blobs) * 65535.0
    lam = np.full((H, W), background, np.float64)
    render_blobs(H, W, cy, cx, s, amp, out=lam)
    counts = np.minimum(rng.poisson(lam), 65535).astype(np.uint16)
    return (counts.astype(np.float32) / np.float32(65535.0)).astype(np.float32)


def batch64(n_frames: int = 64, H: int = 1024, W: int = 1024, first_seed: int = 1000):
    """Uniform batch of 1024x1024 camera frames, blob count U{100..1000}."""
    frames = []
    for f in range(n_frames):
        nb = int(np.random.default_rng(first_seed + f).integers(100, 1001))
        frames.append(camera_frame(first_seed + f + 100000, H, W, n_blobs=nb))
    return frames


def mixed_shapes(n_frames: int = 128, seed: int = 2000):
    """(H, W) of the uneven batch: side S from SIDES, square or (S/2) x S."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(n_frames):
        S = int(rng.choice(SIDES))
        crop = bool(rng.random() < 0.5)
        shapes.append((S // 2, S) if crop else (S, S))
    return shapes


def mixed_frame(f: int, H: int, W: int, first_seed: int = 2000) -> np.ndarray:
    nb = int(round(H * W / 2000.0))
    return camera_frame(first_seed + 1 + f, H, W, n_blobs=nb)


def mixed128(n_frames: int = 128, seed: int = 2000):
    return [mixed_frame(f, H, W, seed) for f, (H, W) in enumerate(mixed_shapes(n_frames, seed))]


def poisson_arrivals(rate: float = 200.0, duration: float = 60.0, seed: int = 3000) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    n_est = int(rate * duration * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, n_est))
    return t[t < duration]


def planted_blob(H: int, W: int, cy: int, cx: int, s: float, amp: float = 1.0) -> np.ndarray:
    """A single noiseless Gaussian blob centred on an integer pixel."""
    return render_blobs(H, W, [cy], [cx], [s], [amp]).astype(np.float32)
