"""Pixel-interleaved (packed HWC) images on the GPU through the C ABI: every
form equals the planar result of the same image bitwise, in place and
pitched/unaligned layouts included."""
import numpy as np
import pytest

import oracle
import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

FORMS = ("fused", "direct", "2pass")


def _torch():
    import torch

    return torch


def run_planar(form, a, k):
    out = gu.nan_like(a)
    if form == "2pass":
        cs.conv_sep5_2pass(a, out, k)
    else:
        cs.conv_sep5_1pass(a, out, k, cs.CONV_1PASS_FUSED if form == "fused" else cs.CONV_1PASS_DIRECT25)
    return out


def run_hwc(form, h, k, out=None):
    """h: [rows, cols, planes] view; returns the output view."""
    out = gu.nan_like(h) if out is None else out
    ii = cs.image_hwc(h)
    assert cs.image_hwc(out).pitch == ii.pitch
    if form == "2pass":
        cs.conv_sep5_2pass(h, out, k, img=ii)
    else:
        cs.conv_sep5_1pass(h, out, k, cs.CONV_1PASS_FUSED if form == "fused" else cs.CONV_1PASS_DIRECT25,
                           img=ii)
    return out


def bits(t):
    torch = _torch()
    return t if t.dtype == torch.float32 else t.view(torch.int16)


SHAPES = [(3, 77, 600), (3, 9, 1031), (2, 130, 257), (4, 40, 300), (3, 300, 12), (4, 5, 5),
          (2, 33, 1030), (3, 6, 170)]


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{p}x{r}x{c}" for p, r, c in SHAPES])
def test_hwc_equals_planar(dtype, shape):
    P, R, C = shape
    host32 = synth.image(1700 + P + R + C, P, R, C)
    host = synth.to_storage(host32, dtype) if dtype != "f32" else host32
    a = gu.to_device(host, dtype)                       # [P, R, C]
    h = a.permute(1, 2, 0).contiguous()                 # [R, C, P]
    k = synth.taps_random(1701 + C)
    torch = _torch()
    for form in FORMS:
        ref = run_planar(form, a, k)
        got = run_hwc(form, h, k)
        assert torch.equal(bits(got.permute(2, 0, 1).contiguous()), bits(ref)), form


def test_hwc_against_oracle():
    P, R, C = 3, 64, 700
    host = synth.image(1800, P, R, C)
    k = synth.taps_random(1801)
    h = gu.to_device(host).permute(1, 2, 0).contiguous()
    got = run_hwc("fused", h, k).permute(2, 0, 1).cpu().numpy()
    gu.check_f32(got, oracle.conv5(host.astype(np.float64), k.astype(np.float64), nthreads=0))


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("P", [2, 3, 4])
def test_hwc_pitched_and_unaligned(dtype, P):
    """Rows padded (pitch > cols*planes) and an offset base: same bits, and
    the padding is untouched."""
    torch = _torch()
    R, C = 37, 211
    host32 = synth.image(1900 + P, P, R, C)
    host = synth.to_storage(host32, dtype) if dtype != "f32" else host32
    a = gu.to_device(host, dtype)
    h = a.permute(1, 2, 0).contiguous()
    k = synth.taps_random(1901)
    for form in FORMS:
        ref = run_hwc(form, h, k)
        for pad, off in ((16, 0), (5, 1)):
            big_in = torch.zeros(R, C * P + pad, dtype=a.dtype, device="cuda")
            big_out = torch.full_like(big_in, 3.0)
            vin = big_in[:, off:off + C * P].view(R, C, P) if off == 0 else \
                big_in[:, off:off + C * P].unflatten(1, (C, P))
            vin.copy_(h)
            vout = big_out[:, off:off + C * P].unflatten(1, (C, P))
            run_hwc(form, vin, k, out=vout)
            assert torch.equal(bits(vout.contiguous()), bits(ref)), (form, pad, off)
            mask = torch.ones_like(big_out, dtype=torch.bool)
            mask[:, off:off + C * P] = False
            assert torch.all(big_out[mask] == 3.0), (form, pad, off)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_hwc_in_place(dtype):
    """out == in: copy-back single pass and in-place two-pass."""
    torch = _torch()
    P, R, C = 3, 50, 400
    host32 = synth.image(2000, P, R, C)
    host = synth.to_storage(host32, dtype) if dtype != "f32" else host32
    h = gu.to_device(host, dtype).permute(1, 2, 0).contiguous()
    k = synth.taps_random(2001)
    for form in FORMS:
        ref = run_hwc(form, h, k)
        b = h.clone()
        run_hwc(form, b, k, out=b)
        assert torch.equal(bits(b), bits(ref)), form


@pytest.mark.parametrize("shape", [(3, 4, 100), (3, 100, 4), (2, 1, 1), (4, 4, 4)])
def test_hwc_tiny_is_zero(shape):
    P, R, C = shape
    h = gu.to_device(synth.image(21, P, R, C) + 1.0).permute(1, 2, 0).contiguous()
    for form in FORMS:
        got = run_hwc(form, h, synth.taps_random(22)).cpu().numpy()
        assert np.all(got == 0) and not np.any(np.signbit(got)), form


def test_hwc_full_hd_rgb():
    """1080 x 1920 RGB FP32 (a video frame): all forms equal the planar result."""
    torch = _torch()
    P, R, C = 3, 1080, 1920
    host = synth.image(2100, P, R, C)
    a = gu.to_device(host)
    h = a.permute(1, 2, 0).contiguous()
    k = synth.taps_random(2101)
    for form in FORMS:
        assert torch.equal(run_hwc(form, h, k).permute(2, 0, 1), run_planar(form, a, k)), form


@pytest.mark.parametrize("C", [4, 8, 252, 256, 260, 512, 516, 1028])
def test_rgb_aligned_strip_widths(C):
    """Three FP32 channels with 16-byte aligned rows (cols a multiple of 4, the
    vector path): widths around strip boundaries, heights with partial last
    bands, dense and as aligned pitched views (padding untouched), in place:
    each equals the planar fused result bitwise, and one height is checked
    against the oracle."""
    torch = _torch()
    P = 3
    for R in (5, 6, 9, 13, 37):
        host = synth.image(2200 + C + R, P, R, C)
        a = gu.to_device(host)
        k = synth.taps_random(2201 + C)
        ref = run_planar("fused", a, k)
        h = a.permute(1, 2, 0).contiguous()
        got = run_hwc("fused", h, k).permute(2, 0, 1).contiguous()
        assert torch.equal(got, ref), (C, R)
        for pad, off in ((16, 0), (32, 8)):
            big_in = torch.zeros(R, C * P + pad, device="cuda")
            big_out = torch.full_like(big_in, 3.0)
            vin = big_in[:, off:off + C * P].unflatten(1, (C, P))
            vin.copy_(h)
            vout = big_out[:, off:off + C * P].unflatten(1, (C, P))
            run_hwc("fused", vin, k, out=vout)
            assert torch.equal(vout.permute(2, 0, 1).contiguous(), ref), (C, R, pad, off)
            mask = torch.ones_like(big_out, dtype=torch.bool)
            mask[:, off:off + C * P] = False
            assert torch.all(big_out[mask] == 3.0), (C, R, pad, off)
        b = h.clone()
        run_hwc("fused", b, k, out=b)
        assert torch.equal(b.permute(2, 0, 1).contiguous(), ref), (C, R, "in place")
        if R == 37:
            gu.check_f32(got.cpu().numpy(),
                         oracle.conv5(host.astype(np.float64), k.astype(np.float64), nthreads=0))
