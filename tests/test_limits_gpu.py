"""Size limits on the GPU: launches of more than 2^20 workgroups (the grid
loop), rows at the 2^30-byte limit, images larger than 4 GiB (64-bit
offsets), and a packed last strip whose row span sits just under the 2^31
offset limit; sampled outputs against the FP64 oracle on crops."""
import gc

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


def crop_ref(host, k, y, xs):
    """Oracle values of output row y at columns xs, from 5 x 5 crops."""
    R, C = host.shape[-2:]
    out = []
    for x in xs:
        if 2 <= y < R - 2 and 2 <= x < C - 2:
            crop = host[0, y - 2:y + 3, x - 2:x + 3].astype(np.float64)[None]
            out.append(oracle.conv5(crop, k.astype(np.float64))[0, 2, 2])
        else:
            out.append(0.0)
    return np.array(out)


def test_more_than_2_20_workgroups():
    """1 x 20000 x 16384 with 1-row bands: 1.28M tiles, so the kernel's grid
    loop runs a second, partial pass (and its XCD chunking a tail)."""
    torch = _torch()
    R, C = 20000, 16384
    host = synth.image(2200, 1, R, C)
    k = synth.taps_random(2201)
    a = gu.to_device(host)
    ref = torch.empty_like(a)
    cs.conv_sep5_1pass(a, ref, k)
    orig = cs.conv_get_tile_cfg(0, 0)
    try:
        cs.conv_set_tile_cfg(0, 0, 1, 1, 0, 8)
        for mode in (cs.CONV_1PASS_FUSED, cs.CONV_1PASS_DIRECT25):
            out = gu.nan_like(a)
            cs.conv_sep5_1pass(a, out, k, mode)
            if mode == cs.CONV_1PASS_FUSED:
                assert torch.equal(out, ref)
            assert torch.isfinite(out).all()
    finally:
        cs.conv_set_tile_cfg(0, 0, orig.rows_per_tile, orig.waves_per_wg, 0, orig.xcd_slabs)
    rng = np.random.default_rng(2202)
    for y in (0, 2, 9999, 19997, 19998):
        xs = [0, 2, 3, 16381, 16382] + [int(v) for v in rng.integers(0, C, 20)]
        got = ref[0, y, xs].cpu().numpy().astype(np.float64)
        r = crop_ref(host, k, y, xs)
        nz = r != 0
        assert np.all(got[~nz] == 0)
        if nz.any():
            assert np.max(np.abs(got[nz] - r[nz]) / np.abs(r[nz])) <= 1e-6
    del a, ref, host
    gc.collect()


def test_row_at_the_byte_limit():
    """Rows of 2^28 - 8 FP32 columns (just under the 2^30-byte row limit):
    2^20 strips in one band."""
    torch = _torch()
    R, C = 5, (1 << 28) - 8
    rng = np.random.default_rng(2300)
    host = rng.random((1, R, C), dtype=np.float32)
    k = synth.taps_random(2301)
    a = gu.to_device(host)
    out = gu.nan_like(a)
    cs.conv_sep5_1pass(a, out, k)
    assert torch.all(out[0, [0, 1, 3, 4], :] == 0)
    xs = [0, 1, 2, 3, 255, 256, 257, (1 << 24) + 1, (1 << 27) + 3, C - 4, C - 3, C - 2, C - 1]
    xs += [int(v) for v in rng.integers(0, C, 40)]
    got = out[0, 2, xs].cpu().numpy().astype(np.float64)
    r = crop_ref(host, k, 2, xs)
    nz = r != 0
    assert np.all(got[~nz] == 0)
    assert np.max(np.abs(got[nz] - r[nz]) / np.abs(r[nz])) <= 1e-6
    del a, out, host
    gc.collect()


def test_image_larger_than_4_gib():
    """1 x 2^21 x 512 FP32 (4 GiB): element offsets pass 2^32 bytes; fused
    and two-pass agree bitwise and sampled rows match the oracle."""
    torch = _torch()
    R, C = 1 << 21, 512
    rng = np.random.default_rng(2400)
    host = rng.random((1, R, C), dtype=np.float32)
    k = synth.taps_random(2401)
    a = gu.to_device(host)
    f = torch.empty_like(a)
    cs.conv_sep5_1pass(a, f, k)
    t = torch.empty_like(a)
    cs.conv_sep5_2pass(a, t, k)
    assert torch.equal(f, t)
    del t
    for y in (2, (1 << 20) + 7, R - 4, R - 3):
        crop = host[:, y - 2:y + 3, :].astype(np.float64)
        r = oracle.conv5(crop, k.astype(np.float64))[0, 2]
        gu.check_f32(f[0, y:y + 1].cpu().numpy(), r[None])
    assert torch.all(f[0, R - 2:] == 0)
    del a, f, host
    gc.collect()


def test_packed_strip_at_the_span_limit():
    """A last strip of 40 columns packed 4 bands to a wave, in rows of
    59,652,256 bytes: the buffer resource of a middle band group spans
    36 rows = 2,147,481,216 bytes, 2,368 below the 2^31 offset limit that
    packing allows, so the packed path's 32-bit row offsets run at their
    largest.  Packed == unpacked bitwise; the packed strip and the first
    strip match the oracle on crops, at the band-group boundaries."""
    torch = _torch()
    C = 256 * 58254 + 40
    R = 72                       # bands of 8: groups of 4 bands = rows 0-31, 32-63, 64-71
    assert 36 * C * 4 == 2147481216
    rng = np.random.default_rng(2500)
    host = rng.random((1, R, C), dtype=np.float32)
    k = synth.taps_random(2501)
    a = gu.to_device(host)
    orig = cs.conv_get_tile_cfg(0, 0).as_dict()
    try:
        cs.conv_set_tile_cfg(0, 0, 8, 1, 0, 8, 1)       # packing on
        p = gu.nan_like(a)
        cs.conv_sep5_1pass(a, p, k)
        cs.conv_set_tile_cfg(0, 0, 8, 1, 0, 8, -1)      # packing off
        u = gu.nan_like(a)
        cs.conv_sep5_1pass(a, u, k)
        torch.cuda.synchronize()
        assert torch.equal(p, u)
    finally:
        cs.conv_set_tile_cfg(0, 0, **orig)
    del u
    xs = list(range(C - 44, C)) + [0, 1, 2, 3, 4, 255, 256, 257]
    for y in (0, 1, 2, 30, 31, 32, 33, 62, 63, 64, 65, 69, 70, 71):
        got = p[0, y, xs].cpu().numpy().astype(np.float64)
        r = crop_ref(host, k, y, xs)
        nz = r != 0
        assert np.all(got[~nz] == 0), y
        if nz.any():
            assert np.max(np.abs(got[nz] - r[nz]) / np.abs(r[nz])) <= 1e-6, y
    del a, p, host
    gc.collect()
