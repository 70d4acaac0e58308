"""Seeded random parity sweep on the GPU: each case draws a storage type, a
layout (dense, pitched, offset/unaligned, row-interleaved 3R x C, packed HWC),
an entry point and its form (fused, direct, two-pass, copy-back, batch, width
n, pyramid level, two-pass with a 16-bit intermediate) and a shape of 1..700
rows and columns, runs it through the C ABI and compares every output element
with the FP64 oracle: FP32 within max(1e-6, (2n+2)u) relative, 16-bit through
the storage gate, the 16-bit intermediate form under its own derived bound,
and the frame exactly +0.0.  The draw is fixed by the case index, so every run checks the
same cases."""
import numpy as np
import pytest

import oracle
import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu
from tests import test_twopass_t16_gpu as t16

pytestmark = pytest.mark.gpu

DTYPES = ("f32", "f16", "bf16")


def _torch():
    import torch

    return torch


def draw(case):
    rng = np.random.default_rng(9000 + case)
    dtype = DTYPES[rng.integers(0, 3)]
    layout = ("dense", "pitched", "offset", "rows3", "hwc")[rng.integers(0, 5)]
    if layout == "hwc":
        entry = ("fused", "direct", "2pass", "copyback")[rng.integers(0, 4)]
        P = int(rng.integers(2, 5))
    else:
        entry = ("fused", "direct", "2pass", "copyback", "batch", "width_n", "pyramid",
                 "2pass_t16")[rng.integers(0, 8)]
        P = 3 if layout == "rows3" else int(rng.integers(1, 4))
    if entry == "pyramid" and layout == "rows3":
        layout = "dense"
    R = int(rng.integers(1, 701))
    C = int(rng.integers(1, 701))
    n = int(rng.choice([1, 3, 5, 7, 9])) if entry == "width_n" else 5
    mode = int(rng.integers(0, 2)) if entry == "width_n" else 0
    return rng, dtype, layout, entry, P, R, C, n, mode


def place(t, layout, rng):
    """A view of a fresh buffer holding t ([P, R, C]) in the given layout,
    and the descriptor that describes it."""
    torch = _torch()
    P, R, C = t.shape
    if layout == "dense":
        v = t.clone()
        return v, cs.image_of(v)
    if layout == "pitched":
        pad = int(rng.integers(1, 10))
        big = torch.zeros(P, R, C + pad, dtype=t.dtype, device=t.device)
        v = big[:, :, :C]
        v.copy_(t)
        return v, cs.image_of(v)
    if layout == "offset":
        off = int(rng.integers(1, 4))
        flat = torch.zeros(P * R * C + off, dtype=t.dtype, device=t.device)
        v = flat[off:].view(P, R, C)
        v.copy_(t)
        return v, cs.image_of(v)
    if layout == "rows3":
        pad = int(rng.integers(0, 6))
        pitch = P * C + pad
        big = torch.zeros(R * pitch, dtype=t.dtype, device=t.device)
        v = big.as_strided((P, R, C), (C, pitch, 1))
        v.copy_(t)
        return v, cs.image_of(v)
    # hwc
    pad = int(rng.integers(0, 6))
    big = torch.zeros(R, C * P + pad, dtype=t.dtype, device=t.device)
    v = big[:, :C * P].unflatten(1, (C, P))
    v.copy_(t.permute(1, 2, 0))
    return v, cs.image_hwc(v)


def like(v, layout):
    """An output buffer of v's layout filled with NaN."""
    torch = _torch()
    if layout == "dense":
        return torch.full_like(v, float("nan"))
    base = v
    while base._base is not None:
        base = base._base
    big = torch.full_like(base, float("nan"))
    return big.as_strided(v.shape, v.stride(), v.storage_offset())


def dense(v, layout):
    return (v.permute(2, 0, 1) if layout == "hwc" else v).contiguous()


@pytest.mark.parametrize("case", range(64))
def test_random_case(case):
    torch = _torch()
    rng, dtype, layout, entry, P, R, C, n, mode = draw(case)
    host32 = synth.image(9100 + case, P, R, C)
    bits = synth.to_storage(host32, dtype) if dtype != "f32" else host32
    a = gu.to_device(bits, dtype)
    A64 = oracle.decode(bits, dtype)
    k = synth.taps_random_n(9200 + case, n)
    print(f"case {case}: {dtype} {layout} {entry} P={P} R={R} C={C} n={n} mode={mode}", flush=True)

    if entry == "2pass_t16":
        tfmt = ("f16", "bf16")[case % 2]
        vin, img = place(a, layout, rng)
        out = like(vin, layout)
        cs.conv_sep5_2pass_ex(vin, out, k, t16.TCODE[tfmt], img=img)
        got = gu.to_host_bits(dense(out, layout))
        ref = oracle.conv5_twopass_t(A64, k.astype(np.float64), tfmt)
        bound, _ = t16.bound_t16(A64, k, tfmt)
        t16.check_t16(got, dtype, ref, bound)
        return
    if entry == "pyramid":
        vin, iin = place(a, layout, rng)
        out = torch.full((P, (R + 1) // 2, (C + 1) // 2), float("nan"), dtype=a.dtype,
                         device=a.device)
        cs.conv_pyr_down(vin, out, k, in_img=iin)
        got, ref = gu.to_host_bits(out), oracle.pyr_down(A64, k.astype(np.float64), nthreads=0)
        margin = 12
    elif entry == "batch":
        vin, img = place(a, layout, rng)
        out = like(vin, layout)
        second = a[:, : max(1, R // 2), :].contiguous()
        out2 = torch.full_like(second, float("nan"))
        cs.conv_sep5_batch([vin, second], [out, out2], [k, k[::-1].copy()],
                           imgs=[img, cs.image_of(second)])
        got = gu.to_host_bits(dense(out, layout))
        ref = oracle.conv5(A64, k.astype(np.float64), nthreads=0)
        ref2 = oracle.conv5(A64[:, : max(1, R // 2), :], k[::-1].astype(np.float64), nthreads=0)
        got2 = gu.to_host_bits(out2)
        if dtype == "f32":
            gu.check_f32(got2, ref2)
        else:
            gu.gate16(got2, ref2, dtype)
        margin = 12
    else:
        vin, img = place(a, layout, rng)
        if entry == "copyback":
            out = vin
        else:
            out = like(vin, layout)
        if entry in ("fused", "direct", "copyback"):
            cs.conv_sep5_1pass(vin, out, k, cs.CONV_1PASS_DIRECT25 if entry == "direct"
                               else cs.CONV_1PASS_FUSED, img=img)
        elif entry == "2pass":
            cs.conv_sep5_2pass(vin, out, k, img=img)
        else:
            cs.conv_sepn_1pass(vin, out, k, mode, img=img)
        got = gu.to_host_bits(dense(out, layout))
        ref = oracle.conv_sep_n(A64, k.astype(np.float64), nthreads=0)
        margin = 2 * n + 2
    if dtype == "f32":
        gu.check_f32(got, ref, tol=max(1e-6, margin * gu.U32))
    else:
        gu.gate16(got, ref, dtype, margin_u=margin)
