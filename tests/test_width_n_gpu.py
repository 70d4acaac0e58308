"""Odd widths n = 1..9 and full (non-separable) n x n kernels on the GPU,
through the C ABI, against the FP64 oracle (Eq. 1 at width n).

Tolerances (FP32 accumulation, positive data and taps): each 1-D filter is a
chain of n roundings, so the separable forms are within (1 + u)^(2n) - 1
~ 2n u of the exact result; the direct form adds one rounding of
K[a][b] = k_a k_b and ceil(log2 n) of the pairwise row sum.  The relative
bound used is max(1e-6, (2n + 2) u).  With signed, non-separable kernels the
error is bounded against the magnitude sum instead:
|got - exact| <= (n + 5) u * sum |K| |A|.
"""
import numpy as np
import pytest

import oracle
import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

WIDTHS = (1, 3, 5, 7, 9)
FUSED, DIRECT = cs.CONV_1PASS_FUSED, cs.CONV_1PASS_DIRECT25


def _torch():
    import torch

    return torch


def tol_n(n):
    return max(1e-6, (2 * n + 2) * gu.U32)


def run_n(form, a, k, out=None):
    """form in {"fused", "direct", "2pass", "full"} ("full": conv_2d_direct
    with K = k as an n x n matrix)."""
    out = gu.nan_like(a) if out is None else out
    if form == "fused":
        cs.conv_sepn_1pass(a, out, k, FUSED)
    elif form == "direct":
        cs.conv_sepn_1pass(a, out, k, DIRECT)
    elif form == "2pass":
        cs.conv_sepn_2pass(a, out, k)
    elif form == "full":
        cs.conv_2d_direct(a, out, k)
    else:
        raise ValueError(form)
    return out


def oracle_sep(host, k, dtype="f32"):
    A = oracle.decode(host, dtype)
    return oracle.conv_sep_n(A, np.asarray(k, np.float32).astype(np.float64), nthreads=0)


def oracle_full(host, K, dtype="f32"):
    A = oracle.decode(host, dtype)
    return oracle.conv_direct_n(A, np.asarray(K, np.float32).astype(np.float64), nthreads=0)


def border_zero_n(got, n):
    r = n // 2
    P, R, C = got.shape
    m = np.ones((R, C), bool)
    if R >= n and C >= n:
        m[r:R - r, r:C - r] = False
    g = got[:, m].astype(np.float64)
    return bool(np.all(g == 0) and not np.any(np.signbit(g)))


SEP_FORMS = ("fused", "direct", "2pass")
SHAPES = [(3, 77, 600), (1, 9, 1031), (2, 130, 257), (1, 300, 12)]


@pytest.mark.parametrize("n", WIDTHS)
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{p}x{r}x{c}" for p, r, c in SHAPES])
def test_separable_widths_f32(n, shape):
    P, R, C = shape
    host = synth.image(200 + n + R, P, R, C)
    k = synth.taps_random_n(300 + n, n)
    a = gu.to_device(host)
    ref = oracle_sep(host, k)
    outs = {f: gu.to_host_bits(run_n(f, a, k)) for f in SEP_FORMS}
    for f in SEP_FORMS:
        e = gu.check_f32(outs[f], ref, tol=tol_n(n))
        assert border_zero_n(outs[f], n), f
        print(f"n={n} {f} {shape}: max rel err {e:.3e}")
    assert np.array_equal(outs["2pass"], outs["fused"]), "2pass and fused must be bitwise equal"


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_width5_matches_width5_kernels_bitwise(dtype):
    """At n = 5 the width-n kernels do exactly the width-5 arithmetic."""
    P, R, C = 3, 70, 700
    bits = synth.to_storage(synth.image(51, P, R, C), dtype) if dtype != "f32" else \
        synth.image(51, P, R, C)
    k = synth.taps_random(52)
    a = gu.to_device(bits, dtype)
    for mode in (FUSED, DIRECT):
        o5 = gu.nan_like(a)
        cs.conv_sep5_1pass(a, o5, k, mode)
        on = gu.nan_like(a)
        cs.conv_sepn_1pass(a, on, k, mode)
        assert np.array_equal(gu.to_host_bits(o5), gu.to_host_bits(on)), mode
    o5 = gu.nan_like(a)
    cs.conv_sep5_2pass(a, o5, k)
    on = gu.nan_like(a)
    cs.conv_sepn_2pass(a, on, k)
    assert np.array_equal(gu.to_host_bits(o5), gu.to_host_bits(on))
    # the full-kernel entry point with K[a][b] = fl32(k_a k_b) is the direct mode
    K = (k.astype(np.float64)[:, None] * k.astype(np.float64)[None, :]).astype(np.float32)
    of = gu.nan_like(a)
    cs.conv_2d_direct(a, of, K)
    od = gu.nan_like(a)
    cs.conv_sepn_1pass(a, od, k, DIRECT)
    assert np.array_equal(gu.to_host_bits(of), gu.to_host_bits(od))


@pytest.mark.parametrize("n", WIDTHS)
def test_full_kernel_signed(n):
    """Non-separable signed K: error within (n + 5) u * sum |K| |A|."""
    P, R, C = 3, 61, 530
    host = (synth.image(400 + n, P, R, C) * 2 - 1).astype(np.float32)
    K = synth.kernel_signed(500 + n, n)
    a = gu.to_device(host)
    got = gu.to_host_bits(run_n("full", a, K)).astype(np.float64)
    ref = oracle_full(host, K)
    mag = oracle.conv_direct_n(np.abs(host.astype(np.float64)),
                               np.abs(K.astype(np.float64)), nthreads=0)
    err = np.abs(got - ref)
    bound = (n + 5) * gu.U32 * mag
    assert np.all(err <= bound), float(np.max(err - bound))
    assert border_zero_n(got, n)
    nz = mag > 0
    print(f"n={n}: max err / magnitude bound = {float(np.max(err[nz] / mag[nz])):.3e}")


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("n", (7, 9))
@pytest.mark.parametrize("rows", (7, 9, 15, 16, 17, 19, 20, 31, 33, 48))
def test_full_kernel_band_heights(dtype, n, rows):
    """The direct n x n form at n >= 7 walks 16-row bands with a ring of input
    rows: heights around the band and ring lengths, one and several strips
    (ragged widths take the element-wise path), in every storage type, against
    the oracle's bound (plus one rounding to 16 bits) and the zero frame."""
    half_ulp = {"f32": 0.0, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}[dtype]
    for P, C in ((2, 197), (1, 600)):
        host32 = (synth.image(1300 + rows, P, rows, C) * 2 - 1).astype(np.float32)
        bits = synth.to_storage(host32, dtype) if dtype != "f32" else host32
        K = synth.kernel_signed(1400 + n, n)
        got = oracle.decode(gu.to_host_bits(run_n("full", gu.to_device(bits, dtype), K)), dtype)
        ref = oracle_full(bits, K, dtype)
        mag = oracle.conv_direct_n(np.abs(oracle.decode(bits, dtype)),
                                   np.abs(K.astype(np.float64)), nthreads=0)
        bound = (n + 5) * gu.U32 * mag * (1 + half_ulp) + half_ulp * np.abs(ref)
        if dtype != "f32":
            bound = bound + 2.0 ** -24
        assert np.all(np.abs(got - ref) <= bound), (P, rows, C)
        assert border_zero_n(got, n), (P, rows, C)


@pytest.mark.parametrize("n", (3, 7, 9))
def test_full_kernel_shift_and_impulse_exact(n):
    """K with a single 1 moves the image (exact); an impulse reproduces K
    turned by 180 degrees (exact: each output is one product)."""
    torch = _torch()
    r = n // 2
    P, R, C = 2, 40, 300
    host = synth.image(600 + n, P, R, C)
    a = gu.to_device(host)
    K = np.zeros((n, n), np.float32)
    K[n - 1, 0] = 1.0
    got = gu.to_host_bits(run_n("full", a, K))
    ref = np.zeros_like(host)
    ref[:, r:R - r, r:C - r] = host[:, n - 1:R - r + r, 0:C - 2 * r]
    assert np.array_equal(got, ref)
    imp = np.zeros((1, 31, 290), np.float32)
    imp[0, 15, 260] = 1.0
    Kf = synth.kernel_signed(700 + n, n)
    got = gu.to_host_bits(run_n("full", gu.to_device(imp), Kf))
    ref = np.zeros_like(imp)
    ref[0, 15 - r:15 + r + 1, 260 - r:260 + r + 1] = Kf[::-1, ::-1]
    assert np.array_equal(got, ref)
    del torch


@pytest.mark.parametrize("n", WIDTHS)
def test_binomial_exact_all_forms(n):
    """m/256 pixels with binomial taps of width n: every FP32 step is exact
    (all partial sums stay below 2^24 units of 2^-(8 + 2(n-1)))."""
    P, R, C = 3, 50, 520
    host = synth.exact_image(800 + n, P, R, C)
    k = synth.taps_binomial_n(n)
    a = gu.to_device(host)
    ref32 = oracle_sep(host, k).astype(np.float32)
    for f in SEP_FORMS:
        assert np.array_equal(gu.to_host_bits(run_n(f, a, k)), ref32), f
    K = np.outer(k.astype(np.float64), k.astype(np.float64)).astype(np.float32)
    assert np.array_equal(gu.to_host_bits(run_n("full", a, K)), ref32)


@pytest.mark.parametrize("n", WIDTHS)
@pytest.mark.parametrize("shape", [(1, 3, 100), (1, 100, 3), (2, 8, 8), (1, 1, 1)])
def test_smaller_than_width_is_zero(n, shape):
    P, R, C = shape
    host = synth.image(9, P, R, C) + 1.0
    a = gu.to_device(host)
    k = synth.taps_random_n(10, n)
    K = synth.kernel_signed(11, n)
    for f in SEP_FORMS + ("full",):
        got = gu.to_host_bits(run_n(f, a, K if f == "full" else k))
        if R >= n and C >= n:
            assert border_zero_n(got, n), f
        else:
            assert np.all(got == 0) and not np.any(np.signbit(got)), f


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("n", (3, 7, 9))
def test_16bit_widths(dtype, n):
    P, R, C = 3, 45, 1100
    host32 = synth.image(900 + n, P, R, C)
    bits = synth.to_storage(host32, dtype)
    k = synth.taps_random_n(901 + n, n)
    a = gu.to_device(bits, dtype)
    ref = oracle_sep(bits, k, dtype)
    outs = {}
    for f in SEP_FORMS:
        outs[f] = gu.to_host_bits(run_n(f, a, k))
        e, n_mid = gu.gate16(outs[f], ref, dtype, margin_u=2 * n + 2)
        print(f"{dtype} n={n} {f}: max rel err {e:.3e}, {n_mid} midpoint cases")
    assert np.array_equal(outs["2pass"], outs["fused"])
    K = synth.kernel_signed(902 + n, n)
    got = oracle.decode(gu.to_host_bits(run_n("full", a, K)), dtype)
    refK = oracle_full(bits, K, dtype)
    mag = oracle.conv_direct_n(np.abs(oracle.decode(bits, dtype)), np.abs(K.astype(np.float64)),
                               nthreads=0)
    # FP32 error bound plus one rounding to the storage format
    half_ulp = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[dtype]
    assert np.all(np.abs(got - refK) <= (n + 5) * gu.U32 * mag * (1 + half_ulp)
                  + half_ulp * np.abs(refK) + 2.0 ** -24)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("n", (3, 7, 9))
def test_unaligned_matches_aligned(dtype, n):
    """Offset base and odd pitch run the element-wise path: same bits."""
    torch = _torch()
    P, R, C = 2, 40, 333
    host32 = synth.image(1000 + n, P, R, C)
    bits = synth.to_storage(host32, dtype) if dtype != "f32" else host32
    a = gu.to_device(bits, dtype)
    k = synth.taps_random_n(1001 + n, n)
    K = synth.kernel_signed(1002 + n, n)
    big_in = torch.zeros(P, R, C + 3, dtype=a.dtype, device="cuda")
    v_in = big_in[:, :, 1:C + 1]
    v_in.copy_(a)
    for f in SEP_FORMS + ("full",):
        taps = K if f == "full" else k
        ref = gu.to_host_bits(run_n(f, a, taps))
        big_out = torch.full_like(big_in, float("nan"))
        v_out = big_out[:, :, 1:C + 1]
        run_n(f, v_in, taps, out=v_out)
        assert np.array_equal(gu.to_host_bits(v_out), ref), f


@pytest.mark.parametrize("n", (3, 7, 9))
def test_copy_back_in_place(n):
    torch = _torch()
    P, R, C = 3, 50, 400
    host = synth.image(1100 + n, P, R, C)
    a = gu.to_device(host)
    k = synth.taps_random_n(1101 + n, n)
    K = synth.kernel_signed(1102 + n, n)
    for f in ("fused", "direct", "full", "2pass"):
        taps = K if f == "full" else k
        ref = run_n(f, a, taps)
        b = a.clone()
        run_n(f, b, taps, out=b)
        assert torch.equal(b, ref), f


@pytest.mark.parametrize("n", (7, 9))
def test_full_size_sampled_rows(n):
    """3 x 4096 x 4096 FP32 at n = 7, 9 (the size the benchmark times): sampled
    rows of the fused form and of a full signed kernel (walking bands: rows at
    band starts and ends) against the oracle on row crops; fused == 2pass."""
    torch = _torch()
    P, R, C = 3, 4096, 4096
    r = n // 2
    host = synth.image(1200 + n, P, R, C)
    k = synth.taps_random_n(1201 + n, n)
    K = synth.kernel_signed(1202 + n, n)
    a = gu.to_device(host)
    fused = run_n("fused", a, k)
    assert torch.equal(fused, run_n("2pass", a, k))
    full = run_n("full", a, K)
    rows = [0, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 1023, 2047, 2048, 4079, 4080, 4090, 4091, 4092, 4095]
    for y in rows:
        if y < r or y >= R - r:
            assert torch.all(fused[:, y, :] == 0) and torch.all(full[:, y, :] == 0)
            continue
        crop = host[:, y - r:y + r + 1, :]
        ref = oracle_sep(crop, k)[:, r, :]
        gu.check_f32(fused[:, y, :].cpu().numpy()[:, None, :], ref[:, None, :], tol=tol_n(n))
        refK = oracle_full(crop, K)[:, r, :]
        mag = oracle.conv_direct_n(np.abs(crop.astype(np.float64)), np.abs(K.astype(np.float64)),
                                   nthreads=0)[:, r, :]
        got = full[:, y, :].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - refK) <= (n + 5) * gu.U32 * mag)
