"""One pyramid level (width-5 blur + 2x decimation) on the GPU, through the
C ABI: bitwise equal to the fused single pass at the sampled pixels, and
against the FP64 oracle (conv5 sampled at even rows and columns)."""
import numpy as np
import pytest

import oracle
import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def out_like(a):
    torch = _torch()
    P, R, C = a.shape
    return torch.full((P, (R + 1) // 2, (C + 1) // 2), float("nan"), dtype=a.dtype, device=a.device)


def bits_of(t):
    torch = _torch()
    return t if t.dtype == torch.float32 else t.view(torch.int16)


SHAPES = [(3, 64, 256), (3, 77, 600), (1, 9, 1031), (2, 130, 257), (1, 300, 12), (3, 5, 5),
          (1, 6, 7), (2, 2049, 513)]


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{p}x{r}x{c}" for p, r, c in SHAPES])
def test_equals_fused_at_sampled_pixels(dtype, shape):
    P, R, C = shape
    host32 = synth.image(1300 + R + C, P, R, C)
    bits = synth.to_storage(host32, dtype) if dtype != "f32" else host32
    a = gu.to_device(bits, dtype)
    k = synth.taps_random(1301 + R)
    full = gu.nan_like(a)
    cs.conv_sep5_1pass(a, full, k)
    o = out_like(a)
    cs.conv_pyr_down(a, o, k)
    torch = _torch()
    assert torch.equal(bits_of(o), bits_of(full[:, ::2, ::2].contiguous()))


@pytest.mark.parametrize("shape", [(3, 256, 256), (2, 61, 517), (1, 33, 1024)])
def test_f32_against_oracle(shape):
    P, R, C = shape
    host = synth.image(1400 + R, P, R, C)
    k = synth.taps_random(1401)
    o = out_like(gu.to_device(host))
    cs.conv_pyr_down(gu.to_device(host), o, k)
    ref = oracle.pyr_down(host.astype(np.float64), k.astype(np.float64), nthreads=0)
    e = gu.check_f32(gu.to_host_bits(o), ref)
    print(f"pyr {shape}: max rel err {e:.3e}")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_16bit_against_oracle(dtype):
    P, R, C = 3, 90, 1030
    bits = synth.to_storage(synth.image(1500, P, R, C), dtype)
    k = synth.taps_random(1501)
    a = gu.to_device(bits, dtype)
    o = out_like(a)
    cs.conv_pyr_down(a, o, k)
    ref = oracle.pyr_down(oracle.decode(bits, dtype), k.astype(np.float64), nthreads=0)
    e, n_mid = gu.gate16(gu.to_host_bits(o), ref, dtype)
    print(f"pyr {dtype}: max rel err {e:.3e}, {n_mid} midpoint cases")


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_pitched_and_unaligned_layouts(dtype):
    """Offset input, pitched output: the element-wise path gives the same bits."""
    torch = _torch()
    P, R, C = 2, 41, 300
    host32 = synth.image(1600, P, R, C)
    bits = synth.to_storage(host32, dtype) if dtype != "f32" else host32
    a = gu.to_device(bits, dtype)
    k = synth.taps_random(1601)
    ref = out_like(a)
    cs.conv_pyr_down(a, ref, k)
    big_in = torch.zeros(P, R, C + 3, dtype=a.dtype, device="cuda")
    v_in = big_in[:, :, 1:C + 1]
    v_in.copy_(a)
    Ro, Co = (R + 1) // 2, (C + 1) // 2
    big_out = torch.full((P, Ro + 1, Co + 5), 7.0, dtype=a.dtype, device="cuda")
    v_out = big_out[:, 1:Ro + 1, 2:Co + 2]
    cs.conv_pyr_down(v_in, v_out, k)
    assert torch.equal(bits_of(v_out.contiguous()), bits_of(ref))
    mask = torch.ones_like(big_out, dtype=torch.bool)
    mask[:, 1:Ro + 1, 2:Co + 2] = False
    assert torch.all(big_out[mask] == 7.0)
    # a pitched output (pitch Co + 14: a multiple of 4 elements)
    big2 = torch.full((P, Ro, Co + 14), 7.0, dtype=a.dtype, device="cuda")
    cs.conv_pyr_down(a, big2[:, :, :Co], k)
    assert torch.equal(bits_of(big2[:, :, :Co].contiguous()), bits_of(ref))
    assert torch.all(big2[:, :, Co:] == 7.0)


@pytest.mark.parametrize("shape", [(1, 4, 100), (1, 100, 4), (3, 1, 1), (2, 4, 4), (1, 5, 4)])
def test_tiny_images_are_zero(shape):
    host = synth.image(17, *shape) + 1.0
    a = gu.to_device(host)
    o = out_like(a)
    cs.conv_pyr_down(a, o, synth.taps_random(18))
    got = gu.to_host_bits(o)
    assert np.all(got == 0) and not np.any(np.signbit(got))


def test_full_size_equals_fused():
    """3 x 4096 x 4096 FP32: the whole level against the fused single pass."""
    torch = _torch()
    host = synth.image(1, 3, 4096, 4096)
    k = synth.taps_random(2)
    a = gu.to_device(host)
    full = torch.empty_like(a)
    cs.conv_sep5_1pass(a, full, k)
    o = out_like(a)
    cs.conv_pyr_down(a, o, k)
    assert torch.equal(o, full[:, ::2, ::2])
    rows = [0, 1, 2, 511, 1024, 2046, 2047]
    crop_ref = {}
    for yo in rows:
        y = 2 * yo
        if 2 <= y < 4096 - 2:
            crop = host[:, y - 2:y + 3, :].astype(np.float64)
            crop_ref[yo] = oracle.conv5(crop, k.astype(np.float64), nthreads=0)[:, 2, ::2]
        else:
            crop_ref[yo] = np.zeros((3, 2048))
    got = o[:, rows, :].cpu().numpy()
    ref = np.stack([crop_ref[y] for y in rows], axis=1)
    gu.check_f32(got, ref)
