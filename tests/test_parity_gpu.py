"""FP32 parity of the HIP path (through the C ABI) with the FP64 oracle."""
import numpy as np
import pytest

import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

FORMS = ("2pass", "fused", "direct")


def _torch():
    import torch

    return torch


def test_small_config_all_forms():
    """3 x 256 x 256 FP32, seed 0, k = [1,4,6,4,1]/16: every form vs the oracle."""
    host = synth.image(0, 3, 256, 256)
    k = synth.taps_binomial()
    a = gu.to_device(host)
    ref = gu.oracle_of(host, k)
    outs = {}
    for form in FORMS:
        outs[form] = gu.to_host_bits(gu.run(form, a, k))
        gu.check_f32(outs[form], ref)
        assert gu.border_is_zero(outs[form])
    assert np.array_equal(outs["2pass"], outs["fused"]), "2pass and fused must be bitwise equal"


def test_exact_binomial_is_bitwise():
    """m/256 pixels with binomial taps: every FP32 operation is exact."""
    host = synth.exact_image(10, 3, 96, 130)
    k = synth.taps_binomial()
    a = gu.to_device(host)
    ref32 = gu.oracle_of(host, k).astype(np.float32)
    for form in FORMS:
        assert np.array_equal(gu.to_host_bits(gu.run(form, a, k)), ref32), form


SHAPES = [(3, 37, 300), (2, 77, 517), (1, 5, 5), (1, 6, 1031), (3, 130, 257), (1, 9, 256),
          (3, 200, 1024), (1, 300, 12), (2, 33, 769), (1, 1000, 8), (1, 7, 1536), (3, 66, 260)]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{p}x{r}x{c}" for p, r, c in SHAPES])
def test_random_taps_ragged_shapes(shape):
    P, R, C = shape
    host = synth.image(100 + R + C, P, R, C)
    k = synth.taps_random(7 + R)
    a = gu.to_device(host)
    ref = gu.oracle_of(host, k)
    outs = {f: gu.to_host_bits(gu.run(f, a, k)) for f in FORMS}
    for f in FORMS:
        gu.check_f32(outs[f], ref)
    assert np.array_equal(outs["2pass"], outs["fused"])


@pytest.mark.parametrize("shape", [(1, 4, 100), (1, 100, 4), (3, 1, 1), (1, 2, 3), (2, 4, 4),
                                   (1, 5, 4), (1, 4, 5)])
def test_tiny_images_are_zero(shape):
    host = synth.image(3, *shape) + 1.0
    a = gu.to_device(host)
    k = synth.taps_random(4)
    for f in FORMS:
        got = gu.to_host_bits(gu.run(f, a, k))
        assert np.all(got == 0) and not np.any(np.signbit(got)), f


def test_every_tile_shape_is_bitwise_identical():
    """Kind 0 (fused, two-pass) and kind 2 (direct 25-tap) configurations."""
    host = synth.image(41, 3, 150, 700)
    k = synth.taps_random(42)
    a = gu.to_device(host)
    orig = cs.conv_get_tile_cfg(0, cs.KIND_IMAGE)
    orig_d = cs.conv_get_tile_cfg(0, cs.KIND_DIRECT)
    try:
        base = {f: gu.to_host_bits(gu.run(f, a, k)) for f in FORMS}
        for th in (1, 3, 4, 8, 16, 17, 64, 200):
            for w in (1, 2, 4):
                for x in (0, 1, 2, 8, 64):
                    cs.conv_set_tile_cfg(0, cs.KIND_IMAGE, th, w, 0, x)
                    cs.conv_set_tile_cfg(0, cs.KIND_DIRECT, th, w, 0, x)
                    for f in FORMS:
                        got = gu.to_host_bits(gu.run(f, a, k))
                        assert np.array_equal(got, base[f]), (th, w, x, f)
    finally:
        cs.conv_set_tile_cfg(0, cs.KIND_IMAGE, **orig.as_dict())
        cs.conv_set_tile_cfg(0, cs.KIND_DIRECT, **orig_d.as_dict())
    gu.check_f32(base["fused"], gu.oracle_of(host, k))
    gu.check_f32(base["direct"], gu.oracle_of(host, k))


def test_pitched_and_offset_layouts():
    """Row pitch and plane stride larger than the image, aligned and unaligned."""
    torch = _torch()
    P, R, C = 3, 61, 340
    host = synth.image(51, P, R, C)
    k = synth.taps_random(52)
    ref = gu.oracle_of(host, k)
    for (pr, pc, r0, c0) in ((5, 64, 0, 0), (3, 37, 1, 3), (0, 4, 0, 4), (2, 1, 1, 1)):
        big_in = torch.zeros(P, R + pr, C + pc, device="cuda")
        big_in[:, r0:r0 + R, c0:c0 + C] = torch.from_numpy(host).cuda()
        big_out = torch.full((P, R + pr, C + pc), 12345.0, device="cuda")
        vin = big_in[:, r0:r0 + R, c0:c0 + C]
        vout = big_out[:, r0:r0 + R, c0:c0 + C]
        for f in FORMS:
            big_out.fill_(12345.0)
            gu.run(f, vin, k, out=vout)
            bo = big_out.cpu().numpy()
            gu.check_f32(bo[:, r0:r0 + R, c0:c0 + C], ref)
            mask = np.ones(bo.shape, bool)
            mask[:, r0:r0 + R, c0:c0 + C] = False
            assert np.all(bo[mask] == 12345.0), (f, pr, pc, "wrote outside the image")


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_unaligned_pointer_matches_aligned(dtype):
    """The element-wise path (misaligned base) is bitwise equal to the vector path."""
    torch = _torch()
    host = synth.image(61, 3, 90, 512)
    k = synth.taps_random(62)
    a = gu.to_device(synth.to_storage(host, dtype), dtype)
    flat = torch.zeros(host.size + 1, dtype=a.dtype, device="cuda")
    flat[1:] = a.reshape(-1)
    au = flat[1:].view(3, 90, 512)          # one-element offset: not 16-byte aligned
    for f in FORMS:
        ref = gu.to_host_bits(gu.run(f, a, k))
        fo = torch.full((host.size + 1,), float("nan"), dtype=a.dtype, device="cuda")
        got = gu.run(f, au, k, out=fo[1:].view(3, 90, 512))
        assert np.array_equal(gu.to_host_bits(got), ref), f


def test_2pass_in_place_and_workspace():
    torch = _torch()
    host = synth.image(71, 3, 128, 384)
    k = synth.taps_random(72)
    a = gu.to_device(host)
    ref = gu.to_host_bits(gu.run("fused", a, k))
    tmp = torch.empty(3 * 128 * 384, device="cuda")
    got = gu.to_host_bits(gu.run("2pass", a, k, tmp=tmp))
    assert np.array_equal(got, ref)
    b = a.clone()
    cs.conv_sep5_2pass(b, b, k)  # the paper's in-place two-pass
    assert np.array_equal(gu.to_host_bits(b), ref)


def test_signed_asymmetric_taps():
    host = synth.image(81, 3, 64, 200) * 2 - 1
    k = synth.taps_signed(82)
    a = gu.to_device(host)
    for f in FORMS:
        gu.check_signed(gu.to_host_bits(gu.run(f, a, k)), host, k)


def test_delta_impulse_gives_rounded_outer_product():
    """B[y0+d][x0+e] = RNE32(k[2-d] k[2-e]) exactly (kernel turned by 180 deg)."""
    host = np.zeros((1, 21, 300), np.float32)
    y0, x0 = 10, 257
    host[0, y0, x0] = 1.0
    k = synth.taps_signed(91)
    a = gu.to_device(host)
    ref32 = gu.oracle_of(host, k).astype(np.float32)
    for f in FORMS:
        assert np.array_equal(gu.to_host_bits(gu.run(f, a, k)), ref32), f


def test_constant_image_constant_interior():
    host = np.full((3, 40, 260), 0.7, np.float32)
    k = synth.taps_random(95)
    a = gu.to_device(host)
    ref = gu.oracle_of(host, k)
    for f in FORMS:
        got = gu.to_host_bits(gu.run(f, a, k))
        inner = got[:, 2:-2, 2:-2]
        assert np.all(inner == inner.flat[0]), f
        gu.check_f32(got, ref)


def test_non_default_stream():
    torch = _torch()
    host = synth.image(97, 3, 100, 640)
    k = synth.taps_random(98)
    a = gu.to_device(host)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = {f: gu.run(f, a, k) for f in FORMS}
    s.synchronize()
    ref = gu.oracle_of(host, k)
    for f in FORMS:
        gu.check_f32(gu.to_host_bits(outs[f]), ref)


def test_full_size_sampled_rows():
    """3 x 4096 x 4096 FP32 (the benchmark workload, default launch config):
    sampled output rows against the oracle, whole image 2pass == fused."""
    torch = _torch()
    P, R, C = 3, 4096, 4096
    host = synth.image(1, P, R, C)
    k = synth.taps_random(2)
    a = gu.to_device(host)
    outs = {f: gu.run(f, a, k) for f in FORMS}
    assert torch.equal(outs["2pass"], outs["fused"])
    rows = [0, 1, 2, 3, 4, 31, 32, 33, 63, 64, 65, 127, 128, 2047, 2048, 2049, 4091, 4092, 4093,
            4094, 4095]
    refs = gu.sample_rows_oracle(host, k, rows)
    for f in ("fused", "direct"):
        got = outs[f][:, rows, :].cpu().numpy()
        ref = np.stack([refs[y] for y in rows], axis=1)
        e = gu.check_f32(got, ref)
        print(f"{f}: max rel err on {len(rows)} sampled rows = {e:.3e}")
    for f in FORMS:
        o = outs[f]
        assert torch.all(o[:, :2, :] == 0) and torch.all(o[:, -2:, :] == 0)
        assert torch.all(o[:, :, :2] == 0) and torch.all(o[:, :, -2:] == 0)
        assert torch.isfinite(o).all()


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_1pass_copy_back_in_place(dtype):
    """out == in: the single-pass with copy-back gives the out-of-place result,
    in place, and touches nothing outside the image (pitched layout)."""
    torch = _torch()
    P, R, C = 3, 70, 520
    host32 = synth.image(111, P, R, C)
    bits = synth.to_storage(host32, dtype)
    k = synth.taps_random(112)
    a = gu.to_device(bits, dtype)
    for mode in (cs.CONV_1PASS_FUSED, cs.CONV_1PASS_DIRECT25):
        ref = gu.nan_like(a)
        cs.conv_sep5_1pass(a, ref, k, mode)
        big = torch.zeros(P, R + 2, C + 8, dtype=a.dtype, device="cuda")
        big.fill_(3.0)
        v = big[:, 1:R + 1, 4:C + 4]
        v.copy_(a)
        cs.conv_sep5_1pass(v, v, k, mode)
        assert torch.equal(v.view(torch.int16) if dtype != "f32" else v,
                           ref.view(torch.int16) if dtype != "f32" else ref), mode
        mask = torch.ones_like(big, dtype=torch.bool)
        mask[:, 1:R + 1, 4:C + 4] = False
        assert torch.all(big[mask] == 3.0)


def test_row_interleaved_3RxC_layout():
    """Each row holds the rows of all three planes (the 3R x C layout of the
    paper's task agglomeration); each plane keeps its own 2-pixel border."""
    torch = _torch()
    P, R, C = 3, 90, 300
    host = synth.image(121, P, R, C)
    k = synth.taps_random(122)
    buf_in = torch.from_numpy(np.ascontiguousarray(host.transpose(1, 0, 2))).cuda()  # [R][3][C]
    vin = buf_in.view(R, P * C).as_strided((P, R, C), (C, P * C, 1))
    ref = gu.oracle_of(host, k)
    for f in FORMS:
        buf_out = torch.full((R, P * C), float("nan"), device="cuda")
        vout = buf_out.as_strided((P, R, C), (C, P * C, 1))
        gu.run(f, vin, k, out=vout)
        got = buf_out.view(R, P, C).permute(1, 0, 2).cpu().numpy()
        gu.check_f32(got, ref)
