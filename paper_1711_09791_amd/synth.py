"""Seeded synthetic inputs for the width-5 separable convolution.

This module only draws inputs; it holds none of the convolution's arithmetic.
Both the HIP path and the FP64 oracle are fed from it.

The paper's test images are not published: it states only that they are
square, 3 colour planes, 1152^2 to 8748^2 (Section 4, Experimental Setup),
and that the kernel is a 5x5 separable Gaussian (Section 4).  The generators
below stand
in for them:

* pixels: uniform [0, 1) FP32 from numpy's PCG64 (multiples of 2^-24);
* taps: the binomial [1, 4, 6, 4, 1] / 16 (a width-5 Gaussian approximation,
  exact in FP32), or positive random taps normalised to sum 1: raw U[0, 1)
  from PCG64, normalised in FP64, then rounded once to FP32 (the FP32 array is
  the kernel of record);
* uneven batches: H and W = 8 * U{30..270} (so 240..2160, multiples of 8);
* serving: exponential inter-arrival times, sizes drawn from four video frames.
"""
from __future__ import annotations

import numpy as np

#: Serving frame sizes (rows, cols), each with 3 colour planes.
SERVE_SIZES = ((480, 640), (720, 1280), (1080, 1920), (2160, 3840))


def image(seed: int, planes: int, rows: int, cols: int) -> np.ndarray:
    """Uniform [0, 1) FP32 image, shape [planes, rows, cols]."""
    rng = np.random.default_rng(seed)
    return rng.random((planes, rows, cols), dtype=np.float32)


def exact_image(seed: int, planes: int, rows: int, cols: int) -> np.ndarray:
    """Pixels m / 256 with m uniform in 0..255 (8-bit image scaled to [0, 1))."""
    rng = np.random.default_rng(seed)
    m = rng.integers(0, 256, size=(planes, rows, cols))
    return (m.astype(np.float32) / np.float32(256.0)).astype(np.float32)


def taps_binomial() -> np.ndarray:
    """[1, 4, 6, 4, 1] / 16 as FP32 (every value exact)."""
    return np.array([1, 4, 6, 4, 1], dtype=np.float64).astype(np.float32) / np.float32(16)


def taps_random(seed: int) -> np.ndarray:
    """Five positive taps normalised to sum 1 in FP64, then rounded to FP32."""
    rng = np.random.default_rng(seed)
    raw = rng.random(5)
    while raw.sum() == 0.0:  # pragma: no cover - probability 0
        raw = rng.random(5)
    return (raw / raw.sum()).astype(np.float32)


def taps_signed(seed: int) -> np.ndarray:
    """Five signed taps uniform in [-1, 1) (for asymmetric/cancellation tests)."""
    rng = np.random.default_rng(seed)
    return (rng.random(5) * 2.0 - 1.0).astype(np.float32)


def taps_binomial_n(n: int) -> np.ndarray:
    """Binomial row n-1 over 2^(n-1) as FP32 (exact for n <= 25)."""
    from math import comb

    return (np.array([comb(n - 1, i) for i in range(n)], dtype=np.float64)
            / 2.0 ** (n - 1)).astype(np.float32)


def taps_random_n(seed: int, n: int) -> np.ndarray:
    """n positive taps normalised to sum 1 in FP64, then rounded to FP32."""
    rng = np.random.default_rng(seed)
    raw = rng.random(n) + 1e-3
    return (raw / raw.sum()).astype(np.float32)


def kernel_signed(seed: int, n: int) -> np.ndarray:
    """A full n x n FP32 kernel with signed entries uniform in [-1, 1) (not
    separable: rank n with probability 1)."""
    rng = np.random.default_rng(seed)
    return (rng.random((n, n)) * 2.0 - 1.0).astype(np.float32)


def batch_shapes(seed: int, n: int) -> list[tuple[int, int]]:
    """n (rows, cols) pairs, each 8 * U{30..270} (240..2160, multiples of 8)."""
    rng = np.random.default_rng(seed)
    hw = rng.integers(30, 271, size=(n, 2)) * 8
    return [(int(h), int(w)) for h, w in hw]


def serving_stream(seed_arrival: int, seed_size: int, n: int, rate_per_s: float,
                   sizes=SERVE_SIZES):
    """Poisson request stream: (arrival offsets in s, (rows, cols) per request),
    sizes drawn uniformly from `sizes`."""
    ra = np.random.default_rng(seed_arrival)
    rs = np.random.default_rng(seed_size)
    gaps = ra.exponential(1.0 / rate_per_s, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    idx = rs.integers(0, len(sizes), size=n)
    return arrivals, [tuple(sizes[i]) for i in idx]


def to_storage(img_f32: np.ndarray, dtype: str) -> np.ndarray:
    """Convert an FP32 image to a storage dtype by round-to-nearest-even.

    Returns float32 for "f32", or raw uint16 bits for "f16" / "bf16"
    (the conversion is torch's CPU cast, which rounds to nearest even).
    """
    if dtype == "f32":
        return np.ascontiguousarray(img_f32, dtype=np.float32)
    import torch

    t = torch.from_numpy(np.ascontiguousarray(img_f32, dtype=np.float32))
    if dtype == "f16":
        t = t.to(torch.float16)
    elif dtype == "bf16":
        t = t.to(torch.bfloat16)
    else:
        raise ValueError(dtype)
    return t.view(torch.int16).numpy().view(np.uint16).copy()
