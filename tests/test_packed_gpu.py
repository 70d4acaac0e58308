"""Packed last strips: an aligned image whose last column strip is narrower
than a wave (64*VEC columns) has that strip cut into a piece of 32 lanes,
taken by one wave for 2 consecutive bands, and pieces of 16 lanes, taken by
one wave for 4 bands (a strip of at most 16 lanes: one 16-lane piece; 17..32:
one 32-lane piece; 33..48: 32 + 16; 49..63: 32 + 16 + 16).  Packing is forced
on (pack_tail = 1) at these small sizes; each case is checked against the
FP64 oracle and bitwise against the same launch with packing off (and the
fused form against the two-pass form), with the pitch padding of the output
left untouched."""
import numpy as np
import pytest

import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

DTYPE_CODE = {"f32": 0, "f16": 1, "bf16": 2}
VEC = {"f32": 4, "f16": 8, "bf16": 8}


def _torch():
    import torch

    return torch


@pytest.fixture
def restore_cfg():
    saved = {(d, kd): cs.conv_get_tile_cfg(d, kd).as_dict() for d in range(3) for kd in (0, 1, 2)}
    yield
    for (d, kd), c in saved.items():
        cs.conv_set_tile_cfg(d, kd, c["rows_per_tile"], c["waves_per_wg"],
                             c["persist_wgs_per_cu"], c["xcd_slabs"], c["pack_tail"])


def widths(dtype):
    """Widths whose last strip is cut into each set of pieces (16; 32; 32+16;
    32+16+16 lanes) at both ends of their ranges, a full last strip, and
    single-strip images."""
    v = VEC[dtype]
    sw = 64 * v
    return [16 * v, 16 * v - v, 32 * v, 17 * v, sw + v, sw + 16 * v, 2 * sw + 32 * v,
            2 * sw + 33 * v, 5 * v, v, 40 * v, sw + 48 * v, 49 * v, 2 * sw + 63 * v, sw + 56 * v,
            2 * sw]


def set_kind0_and_direct(dtype, th, pack, x=8):
    """The same tile configuration for the fused (kind 0) and direct (kind 2) kernels."""
    cs.conv_set_tile_cfg(DTYPE_CODE[dtype], cs.KIND_IMAGE, th, 1, 0, x, pack)
    cs.conv_set_tile_cfg(DTYPE_CODE[dtype], cs.KIND_DIRECT, th, 1, 0, x, pack)


def pitched(t, pad):
    """A view of t in a buffer with `pad` extra elements per row, padding = 7."""
    torch = _torch()
    P, R, C = t.shape
    big = torch.full((P, R, C + pad), 7.0, dtype=t.dtype, device=t.device)
    v = big[:, :, :C]
    v.copy_(t)
    return big, v


def check(dtype, got_bits, host_bits, k, margin=12):
    ref = gu.oracle_of(host_bits, k, dtype)
    if dtype == "f32":
        gu.check_f32(got_bits, ref)
    else:
        gu.gate16(got_bits, ref, dtype, margin_u=margin)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("th", [4, 8])
def test_single_image_packed_strips(dtype, th, restore_cfg):
    torch = _torch()
    set_kind0_and_direct(dtype, th, 1)
    v = VEC[dtype]
    for i, C in enumerate(widths(dtype)):
        # heights: partial last band, partial last group of bands, one band
        for R in (th * 4 + 3, th * 5, th * 2 + 1, 2 * th - 1, 97):
            P = 1 + (i + R) % 3
            host = synth.to_storage(synth.image(5000 + 7 * i + R, P, R, C), dtype)
            a = gu.to_device(host, dtype)
            k = synth.taps_random(5100 + i)
            pad = v * (1 + i % 3)
            buf_f, out_f = pitched(gu.nan_like(a), pad)
            ain_big, ain = pitched(a, pad)
            cs.conv_sep5_1pass(ain, out_f, k, cs.CONV_1PASS_FUSED)
            two = gu.run("2pass", a, k)
            got = gu.to_host_bits(out_f.contiguous())
            check(dtype, got, host, k)
            assert np.array_equal(got, gu.to_host_bits(two)), (dtype, th, P, R, C)
            assert torch.all(buf_f[:, :, C:] == 7.0), "pitch padding was written"
            # direct25 (packed for FP32 only) vs the same launch unpacked
            buf_d, out_d = pitched(gu.nan_like(a), pad)
            cs.conv_sep5_1pass(ain, out_d, k, cs.CONV_1PASS_DIRECT25)
            set_kind0_and_direct(dtype, th, -1)
            ref_d = gu.run("direct", a, k)
            set_kind0_and_direct(dtype, th, 1)
            got_d = gu.to_host_bits(out_d.contiguous())
            check(dtype, got_d, host, k)
            assert np.array_equal(got_d, gu.to_host_bits(ref_d)), (dtype, th, P, R, C)
            assert torch.all(buf_d[:, :, C:] == 7.0), "pitch padding was written"


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_copy_back_packed(dtype, restore_cfg):
    """In-place single pass (scratch with cached stores, then the copy)."""
    cs.conv_set_tile_cfg(DTYPE_CODE[dtype], 0, 8, 1, 0, 8, 1)
    v = VEC[dtype]
    for C in (16 * v, 64 * v + 20 * v):
        host = synth.to_storage(synth.image(5200 + C, 3, 75, C), dtype)
        a = gu.to_device(host, dtype)
        k = synth.taps_random(5201)
        ref = gu.to_host_bits(gu.run("2pass", a, k))
        cs.conv_sep5_1pass(a, a, k, cs.CONV_1PASS_FUSED)
        assert np.array_equal(gu.to_host_bits(a), ref)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("mode", [cs.CONV_1PASS_FUSED, cs.CONV_1PASS_DIRECT25])
def test_batch_packed_strips(dtype, mode, restore_cfg):
    """Batch of aligned images with narrow last strips (the aligned-only batch
    kernel), the same batch with one unaligned image (the general kernel),
    and one with more images than the kernel argument holds: each equals the
    single-image launches with packing off."""
    torch = _torch()
    v = VEC[dtype]
    shapes = [(37, 16 * v), (64, 64 * v + 8 * v), (9, 32 * v), (130, 2 * 64 * v + 24 * v),
              (17, 5 * v), (40, 64 * v), (23, 64 * v + 40 * v)]
    hosts = [synth.to_storage(synth.image(5300 + i, 3, h, w), dtype) for i, (h, w) in enumerate(shapes)]
    ks = [synth.taps_random(5400 + i) for i in range(len(shapes))]
    ins = [gu.to_device(h, dtype) for h in hosts]
    # references: single-image launches with packing off
    cs.conv_set_tile_cfg(DTYPE_CODE[dtype], 0, 8, 1, 0, 8, -1)
    refs = []
    for a, k in zip(ins, ks):
        o = gu.nan_like(a)
        cs.conv_sep5_1pass(a, o, k, mode)
        refs.append(gu.to_host_bits(o))
    for variant in ("aligned", "one_unaligned", "descriptor_table"):
        bins, bks, brefs, bhosts = list(ins), list(ks), list(refs), list(hosts)
        if variant == "descriptor_table":
            # more images than ride in the kernel argument (inputs shared)
            bins, bks, brefs, bhosts = bins * 3, bks * 3, brefs * 3, bhosts * 3
        if variant == "one_unaligned":
            h = synth.to_storage(synth.image(5500, 2, 41, 16 * v + 3), dtype)
            bhosts.append(h)
            bins.append(gu.to_device(h, dtype))
            bks.append(synth.taps_random(5501))
            o = gu.nan_like(bins[-1])
            cs.conv_sep5_1pass(bins[-1], o, bks[-1], mode)
            brefs.append(gu.to_host_bits(o))
        for th in (4, 8):
            cs.conv_set_tile_cfg(DTYPE_CODE[dtype], 1, th, 1, 0, 8, 1)
            outs = [gu.nan_like(a) for a in bins]
            cs.conv_sep5_batch(bins, outs, bks, mode=mode)
            torch.cuda.synchronize()
            for j, (o, r, h, k) in enumerate(zip(outs, brefs, bhosts, bks)):
                got = gu.to_host_bits(o)
                assert np.array_equal(got, r), (variant, th, j)
            check(dtype, gu.to_host_bits(outs[1]), bhosts[1], bks[1])


def test_packed_every_tile_order(restore_cfg):
    """Packing with every XCD order (launch order, slabs, chunks of 2..64 band
    rows) and, for batches, persistent grids: bitwise equal to packing off."""
    torch = _torch()
    host = synth.image(5600, 3, 203, 4 * 64 * 4 + 36)       # FP32: last strip 36 columns
    a = gu.to_device(host)
    k = synth.taps_random(5601)
    set_kind0_and_direct("f32", 8, -1)
    ref = gu.run("fused", a, k)
    ref_d = gu.run("direct", a, k)
    for x in (0, 1, 2, 3, 4, 16, 64):
        for th in (4, 8):
            set_kind0_and_direct("f32", th, 1, x)
            assert torch.equal(gu.run("fused", a, k), ref), (x, th)
            assert torch.equal(gu.run("direct", a, k), ref_d), (x, th)
    for C in (4 * 64 * 4 + 4 * 40, 3 * 64 * 4 + 4 * 60):   # last strip 40 and 60 lanes
        host = synth.image(5602 + C, 3, 203, C)
        b = gu.to_device(host)
        set_kind0_and_direct("f32", 8, -1)
        ref, ref_d = gu.run("fused", b, k), gu.run("direct", b, k)
        for x in (0, 1, 2, 3, 4, 16, 64):
            for th in (4, 8):
                set_kind0_and_direct("f32", th, 1, x)
                assert torch.equal(gu.run("fused", b, k), ref), (C, x, th)
                assert torch.equal(gu.run("direct", b, k), ref_d), (C, x, th)
        gu.check_f32(gu.to_host_bits(ref), gu.oracle_of(host, k))
    shapes = [(70, 256 + 20), (33, 512 + 100), (129, 60), (41, 1024 + 8), (57, 512 + 160),
              (90, 1024 + 232)]
    ins = [gu.to_device(synth.image(5610 + i, 3, h, w)) for i, (h, w) in enumerate(shapes)]
    ks = [synth.taps_random(5620 + i) for i in range(len(shapes))]
    cs.conv_set_tile_cfg(0, 1, 8, 1, 0, 8, -1)
    refs = [gu.nan_like(t) for t in ins]
    cs.conv_sep5_batch(ins, refs, ks)
    for p in (0, 4, 16):
        for x in (0, 1, 2, 8):
            cs.conv_set_tile_cfg(0, 1, 8, 1, p, x, 1)
            outs = [gu.nan_like(t) for t in ins]
            cs.conv_sep5_batch(ins, outs, ks)
            for j, (o, r) in enumerate(zip(outs, refs)):
                assert torch.equal(o, r), (p, x, j)
