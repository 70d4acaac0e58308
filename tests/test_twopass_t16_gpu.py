"""Two-pass form with a 16-bit intermediate (conv_sep5_2pass_ex) against its
own oracle, oracle.conv5_twopass_t: exact row pass, one RNE rounding of each
intermediate value, exact column pass.

Tolerance, derived from the arithmetic.  The GPU rounds its FP32 row chain
t32 (five roundings: |t32 - t| <= 5u sum_j |k_j||A_j|) instead of the exact
t, so an intermediate can differ from the oracle's by one 16-bit unit only
where t lies within that distance of a 16-bit rounding midpoint ("ambiguous"
positions, found here from the exact t); elsewhere it is the oracle's value.
The column chain adds at most 5u sum_a |k_a||T_a|.  So per output pixel

    |g - r| <= sum_a |k_a| delta_a + 5u sum_a |k_a| (|T16_a| + delta_a)

with delta_a one 16-bit unit at ambiguous positions and 0 elsewhere, plus half
a unit of the output format (at the larger magnitude) for 16-bit storage.
"""
import numpy as np
import pytest

import oracle
import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
FMT = {"f16": (10, -14), "bf16": (7, -126)}     # fraction bits, min normal exponent
TCODE = {"f16": cs.CONV_F16, "bf16": cs.CONV_BF16}


def _torch():
    import torch

    return torch


def _ulp(x, fmt):
    mb, emin = FMT[fmt]
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    return np.ldexp(1.0, (np.maximum(e, emin) - mb).astype(np.int64))


def bound_t16(A64, k, tfmt):
    """Per-pixel bound of |GPU - oracle| for the FP32 result (see above)."""
    k = np.asarray(k, dtype=np.float32).astype(np.float64)
    P, R, C = A64.shape
    T = np.zeros_like(A64)
    S = np.zeros_like(A64)                          # sum_j |k_j||A_j|
    for b in range(5):
        T[:, :, 2:C - 2] += k[b] * A64[:, :, b:C - 4 + b]
        S[:, :, 2:C - 2] += abs(k[b]) * np.abs(A64[:, :, b:C - 4 + b])
    ulp = _ulp(T, tfmt)
    frac = np.abs(T) / ulp - np.floor(np.abs(T) / ulp)
    dist = ulp * np.abs(frac - 0.5)                 # to the nearest rounding midpoint
    amb = (T != 0) & (dist <= 5.01 * U * S)
    delta = np.where(amb, ulp, 0.0)
    T16 = oracle.decode(oracle.round_to(T, tfmt), tfmt)
    B = np.zeros_like(A64)
    if R >= 5 and C >= 5:
        for a in range(5):
            sl = slice(a, R - 4 + a)
            B[:, 2:R - 2, 2:C - 2] += abs(k[a]) * (delta[:, sl, 2:C - 2] + 5.01 * U *
                                                   (np.abs(T16[:, sl, 2:C - 2]) + delta[:, sl, 2:C - 2]))
    return B, int(amb.sum())


def check_t16(got_bits, dtype, ref, bound):
    g = oracle.decode(got_bits, dtype)
    assert np.all(np.isfinite(g))
    z = ref == 0
    assert np.all(g[z] == 0) and not np.any(np.signbit(g[z])), "frame must be +0.0"
    err = np.abs(g - ref)
    allow = bound + 1e-300
    if dtype != "f32":
        m = np.maximum(np.abs(ref) + bound, np.abs(g))
        allow = allow + 0.5 * _ulp(m, dtype)
    bad = err > allow
    assert not bad.any(), (int(bad.sum()), float(err[bad].max()), float(allow[bad].min()))


def _run(a, k, tfmt, tmp=None):
    out = gu.nan_like(a)
    cs.conv_sep5_2pass_ex(a, out, k, TCODE[tfmt], d_tmp=tmp)
    return out


SHAPES = [(3, 37, 300), (2, 77, 517), (1, 5, 5), (3, 130, 257), (1, 9, 1031), (2, 200, 1024),
          (1, 4, 9), (3, 66, 260)]


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("tfmt", ["f16", "bf16"])
def test_against_oracle(dtype, tfmt):
    n_amb = 0
    for i, (P, R, C) in enumerate(SHAPES):
        bits = synth.to_storage(synth.image(6000 + i, P, R, C), dtype)
        a = gu.to_device(bits, dtype)
        k = synth.taps_random(6100 + i)
        A64 = oracle.decode(bits, dtype)
        ref = oracle.conv5_twopass_t(A64, k.astype(np.float64), tfmt)
        bound, amb = bound_t16(A64, k, tfmt)
        n_amb += amb
        got = gu.to_host_bits(_run(a, k, tfmt))
        check_t16(got, dtype, ref, bound)
    # ambiguous intermediates are rare (about 10u / unit of them: ~1e-3 for
    # FP16, ~1e-4 for BF16), so nearly every output meets the FP32 bound alone
    assert n_amb < 3e-3 * sum(P * R * C for P, R, C in SHAPES)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("tfmt", ["f16", "bf16"])
def test_exact_intermediates_bitwise(dtype, tfmt):
    """Pixels 0..3 with binomial taps: every intermediate is a multiple of 1/16
    below 4, exact in both 16-bit formats, so the GPU matches the oracle
    exactly (16-bit outputs: its one rounding)."""
    rng = np.random.default_rng(6200)
    host = rng.integers(0, 4, size=(3, 45, 270)).astype(np.float32)
    bits = synth.to_storage(host, dtype)
    a = gu.to_device(bits, dtype)
    k = synth.taps_binomial()
    ref = oracle.conv5_twopass_t(oracle.decode(bits, dtype), k.astype(np.float64), tfmt)
    got = gu.to_host_bits(_run(a, k, tfmt))
    if dtype == "f32":
        assert np.array_equal(got.astype(np.float64), ref)
    else:
        assert np.array_equal(got, oracle.round_to(ref, dtype))


def test_forms_agree():
    """In place == out of place; caller workspace == library memory;
    CONV_F32 == conv_sep5_2pass bitwise; the 16-bit forms differ from the
    FP32 one (the rounding is there)."""
    torch = _torch()
    host = synth.image(6300, 3, 150, 700)
    a = gu.to_device(host)
    k = synth.taps_random(6301)
    for tfmt in ("f16", "bf16"):
        o1 = _run(a, k, tfmt)
        tmp = torch.empty(3 * 150 * 700, dtype=torch.float16, device="cuda")
        o2 = _run(a, k, tfmt, tmp=tmp)
        b = a.clone()
        cs.conv_sep5_2pass_ex(b, b, k, TCODE[tfmt])
        assert torch.equal(o1, o2) and torch.equal(o1, b), tfmt
        assert not torch.equal(o1, gu.run("2pass", a, k))
    f = gu.nan_like(a)
    cs.conv_sep5_2pass_ex(a, f, k, cs.CONV_F32)
    assert torch.equal(f, gu.run("2pass", a, k))


def test_tile_shapes_bitwise():
    """Rows per tile and XCD order do not change the result."""
    torch = _torch()
    host = synth.image(6400, 2, 133, 777)
    a = gu.to_device(host)
    k = synth.taps_random(6401)
    orig = cs.conv_get_tile_cfg(0, 0).as_dict()
    try:
        ref = _run(a, k, "f16")
        for th in (4, 8, 16, 5):
            for x in (0, 1, 8):
                cs.conv_set_tile_cfg(0, 0, th, 2, 0, x)     # waves are forced to 1
                assert torch.equal(_run(a, k, "f16"), ref), (th, x)
    finally:
        cs.conv_set_tile_cfg(0, 0, **orig)


def test_large_image_sampled_rows():
    """3 x 4096 x 4096 FP32 with an FP16 intermediate, in the benchmark's
    configuration: sampled output rows against the oracle on crops (row y
    depends on input rows y-2 .. y+2 only)."""
    host = synth.image(1, 3, 4096, 4096)
    a = gu.to_device(host)
    k = synth.taps_random(2)
    got = gu.to_host_bits(_run(a, k, "f16"))
    rows = [0, 1, 2, 3, 7, 8, 9, 1000, 2047, 2048, 4092, 4093, 4094, 4095]
    for y in rows:
        if y < 2 or y >= 4094:
            assert np.all(got[:, y, :] == 0)
            continue
        crop = host[:, y - 2:y + 3, :].astype(np.float64)
        ref = oracle.conv5_twopass_t(crop, k.astype(np.float64), "f16")[:, 2:3, :]
        bound, _ = bound_t16(crop, k, "f16")
        check_t16(got[:, y:y + 1, :], "f32", ref, bound[:, 2:3, :])
