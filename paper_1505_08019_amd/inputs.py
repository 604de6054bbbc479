"""Seeded synthetic inputs shared by the tests, the benchmark and the load generator.

This module holds no FFT arithmetic: it only draws pixels, shapes and arrival
traces.  Both the GPU path and the FP64 oracle are fed from it, so that the two
sides always see the same bytes.

Recipes (the paper's test images are "gray images" of 128x128 .. 2048x2048,
content unstated, sec. 4; none are available, so these stand in for them):

* ``uniform``: i.i.d. integer pixels in [0, 255] cast to float32, imaginary
  part 0.
* ``smooth``: the sum of 32 isotropic 2D Gaussians (centre uniform over the
  image, sigma uniform in [5, 100] px, amplitude uniform in [0, 255]) plus
  uniform noise in [-2, 2]; not clipped; imaginary part 0.
* ragged batch: side exponents uniform over {6..11} (64..2048 px); a quarter of
  the images rectangular, their width exponent redrawn until it differs.
* serve trace: Poisson arrivals, square sides with exponents uniform over
  {6..12} (64..4096 px), precision class 50/50, cutoff uniform in [0.05, 0.5].

Every generator is ``numpy.random.default_rng(SeedSequence([cfg_seed, index]))``.
"""
from __future__ import annotations

import numpy as np

PREC_FP32 = 0
PREC_SPLIT_BF16 = 1
PREC_FP16 = 2


def rng(cfg_seed: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg_seed), int(index)]))


def uniform_pixels(rows: int, cols: int, cfg_seed: int = 1, index: int = 0) -> np.ndarray:
    """rows x cols complex64 image: integer pixels 0..255 in the real part."""
    g = rng(cfg_seed, index)
    re = g.integers(0, 256, size=(rows, cols)).astype(np.float32)
    out = np.zeros((rows, cols), dtype=np.complex64)
    out.real = re
    return out


def smooth_image(rows: int, cols: int, cfg_seed: int = 2, index: int = 0, n_blobs: int = 32) -> np.ndarray:
    """rows x cols complex64 image: 32 Gaussian blobs plus +-2 uniform noise."""
    g = rng(cfg_seed, index)
    cy = g.uniform(0, rows, size=n_blobs)
    cx = g.uniform(0, cols, size=n_blobs)
    sig = g.uniform(5.0, 100.0, size=n_blobs)
    amp = g.uniform(0.0, 255.0, size=n_blobs)
    yy = np.arange(rows, dtype=np.float64)
    xx = np.arange(cols, dtype=np.float64)
    img = np.zeros((rows, cols), dtype=np.float32)
    for b in range(n_blobs):
        gy = np.exp(-((yy - cy[b]) ** 2) / (2.0 * sig[b] ** 2)) * amp[b]
        gx = np.exp(-((xx - cx[b]) ** 2) / (2.0 * sig[b] ** 2))
        img += np.outer(gy, gx).astype(np.float32)
    img += g.uniform(-2.0, 2.0, size=(rows, cols)).astype(np.float32)
    out = np.zeros((rows, cols), dtype=np.complex64)
    out.real = img
    return out


def image(kind: str, rows: int, cols: int, cfg_seed: int, index: int = 0) -> np.ndarray:
    if kind == "uniform":
        return uniform_pixels(rows, cols, cfg_seed, index)
    if kind == "smooth":
        return smooth_image(rows, cols, cfg_seed, index)
    raise ValueError("unknown image kind %r" % kind)


def ragged_shapes(n: int = 512, cfg_seed: int = 4, min_exp: int = 6, max_exp: int = 11,
                  rect_fraction: float = 0.25) -> list[tuple[int, int]]:
    """Shapes of a ragged batch: power-of-two sides, log-uniform, some rectangular."""
    g = rng(cfg_seed, 0)
    shapes = []
    for _ in range(n):
        er = int(g.integers(min_exp, max_exp + 1))
        ec = er
        if g.uniform() < rect_fraction:
            while ec == er:
                ec = int(g.integers(min_exp, max_exp + 1))
        shapes.append((1 << er, 1 << ec))
    return shapes


def poisson_trace(rate: float, n: int, cfg_seed: int = 5, min_exp: int = 6, max_exp: int = 12) -> dict:
    """Arrival trace of image-filter requests.

    Returns arrays: ``t`` arrival time in seconds (Poisson process of the given
    rate), ``side`` square image side, ``precision`` class (0 FP32 / 1 split
    BF16, 50/50), ``cutoff`` (uniform 0.05..0.5 of Nyquist).
    """
    g = rng(cfg_seed, int(rate))
    gaps = g.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    side = 1 << g.integers(min_exp, max_exp + 1, size=n)
    precision = g.integers(0, 2, size=n)
    cutoff = g.uniform(0.05, 0.5, size=n)
    return {"t": t, "side": side.astype(np.int64), "precision": precision.astype(np.int64),
            "cutoff": cutoff}
