"""Helpers for the GPU tests: device tensors, calls through the C ABI, and the
comparison rules against the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle
import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth

U32 = 2.0 ** -24  # FP32 unit roundoff

TORCH_DT = {"f32": "float32", "f16": "float16", "bf16": "bfloat16"}


def to_device(host: np.ndarray, dtype: str = "f32"):
    """Host image (float32 values, or uint16 bits for 16-bit types) -> GPU tensor."""
    import torch

    if dtype == "f32":
        return torch.from_numpy(np.ascontiguousarray(host, dtype=np.float32)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(host).view(np.int16)).cuda()
    return t.view(getattr(torch, TORCH_DT[dtype]))


def to_host_bits(t) -> np.ndarray:
    """GPU tensor -> float32 values (f32) or raw uint16 bits (16-bit types)."""
    import torch

    t = t.detach().cpu().contiguous()
    if t.dtype == torch.float32:
        return t.numpy()
    return t.view(torch.int16).numpy().view(np.uint16)


def nan_like(t):
    import torch

    return torch.full_like(t, float("nan"))


def run(kind: str, a, k, out=None, tmp=None, stream=None):
    """kind in {"2pass", "fused", "direct"}; returns the output tensor (prefilled NaN)."""
    out = nan_like(a) if out is None else out
    if kind == "2pass":
        cs.conv_sep5_2pass(a, out, k, d_tmp=tmp, stream=stream)
    elif kind == "fused":
        cs.conv_sep5_1pass(a, out, k, cs.CONV_1PASS_FUSED, stream=stream)
    elif kind == "direct":
        cs.conv_sep5_1pass(a, out, k, cs.CONV_1PASS_DIRECT25, stream=stream)
    else:
        raise ValueError(kind)
    return out


def oracle_of(host: np.ndarray, k, dtype: str = "f32") -> np.ndarray:
    """FP64 oracle on the exactly decoded storage values."""
    A = oracle.decode(host, dtype)
    return oracle.conv5(A, np.asarray(k, dtype=np.float32).astype(np.float64), nthreads=0)


def check_f32(got: np.ndarray, ref: np.ndarray, tol: float = 1e-6) -> float:
    """Max elementwise relative error; zeros of the reference must be exact +0."""
    g = got.astype(np.float64)
    assert g.shape == ref.shape
    assert np.all(np.isfinite(g)), "non-finite output (unwritten pixels?)"
    z = ref == 0
    assert np.all(g[z] == 0), "pixels with a zero reference are not zero"
    assert not np.any(np.signbit(g[z])), "zero pixels must be +0.0"
    if np.all(z):
        return 0.0
    e = float(np.max(np.abs(g[~z] - ref[~z]) / np.abs(ref[~z])))
    assert e <= tol, f"max relative error {e:.3e} > {tol:.1e}"
    return e


def gate16(got_bits: np.ndarray, ref: np.ndarray, dtype: str, margin_u: float = 12):
    """16-bit storage gate: the output equals the oracle's exact result rounded
    once to `dtype` (RNE), or is the neighbouring value where the exact result
    lies within the FP32 path's error bound (margin_u * u * |r|) of the
    rounding midpoint.  Returns (max relative error vs the unrounded oracle,
    count of midpoint cases)."""
    ref_bits = oracle.round_to(ref, dtype)
    bad = got_bits != ref_bits
    n_mid = 0
    if np.any(bad):
        g = got_bits[bad].astype(np.int64)
        rb = ref_bits[bad].astype(np.int64)
        assert np.all(np.abs(g - rb) == 1), "output differs by more than one unit"
        gv = oracle.decode(got_bits[bad], dtype)
        rv = oracle.decode(ref_bits[bad], dtype)
        mid = (gv + rv) / 2
        r = ref[bad]
        assert np.all(np.abs(r - mid) <= margin_u * U32 * np.abs(r)), "not a midpoint case"
        n_mid = int(bad.sum())
    got = oracle.decode(got_bits, dtype)
    z = ref == 0
    assert np.all(got[z] == 0)
    e = float(np.max(np.abs(got[~z] - ref[~z]) / np.abs(ref[~z]))) if np.any(~z) else 0.0
    return e, n_mid


def border_is_zero(got: np.ndarray) -> bool:
    P, R, C = got.shape
    m = np.ones((R, C), bool)
    if R >= 5 and C >= 5:
        m[2:R - 2, 2:C - 2] = False
    return bool(np.all(got[:, m] == 0) and not np.any(np.signbit(got[:, m].astype(np.float64))))


def check_signed(got: np.ndarray, host: np.ndarray, k) -> None:
    """Signed taps: |g - r| <= 12 u * sum |k_i k_j| |A| (cancellation-safe bound)."""
    k64 = np.asarray(k, dtype=np.float32).astype(np.float64)
    ref = oracle.conv5(host.astype(np.float64), k64, nthreads=0)
    mag = oracle.conv5(np.abs(host.astype(np.float64)), np.abs(k64), nthreads=0)
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= 12 * U32 * mag + 1e-300), float(np.max(err - 12 * U32 * mag))


def sample_rows_oracle(host: np.ndarray, k, rows, dtype: str = "f32"):
    """Oracle on crops: exact reference for the given output rows only.

    For output row y the 5x5 neighbourhoods lie in input rows y-2..y+2, so the
    oracle on the crop [y-2, y+3) gives row y exactly (column border included).
    Returns {y: reference row [planes, cols]}.
    """
    P, R, C = host.shape
    out = {}
    for y in rows:
        if y < 2 or y >= R - 2:
            out[y] = np.zeros((P, C))
            continue
        crop = host[:, y - 2:y + 3, :]
        out[y] = oracle_of(crop, k, dtype)[:, 2, :]
    return out


def image_f32(seed, P, R, C):
    return synth.image(seed, P, R, C)
