"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before any HIP call."""
import ctypes
import json
import os
import re

import pytest

import paper_1711_09791_amd as cs
from paper_1711_09791_amd import conv_image

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "conv_sep5.h")

pytestmark = pytest.mark.skipif(not os.path.exists(cs.LIB_PATH),
                                reason="libconvsep5.so not built")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(conv_[a-z0-9_]+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("conv_sep5_2pass", "conv_sep5_1pass", "conv_sep5_batch",
                     "conv_serve_submit", "conv_serve_poll", "conv_last_error"):
        assert required in names
    assert set(names) == set(cs.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = cs.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert "gfx950" in cs.conv_version()


def test_loadgen_library_exports_its_header():
    hdr = os.path.join(ROOT, "include", "conv_loadgen.h")
    names = declared_functions(hdr)
    assert set(names) == set(cs.LOADGEN_EXPORTS)
    G = cs.loadgen_lib()
    for name in names:
        assert hasattr(G, name), name
    # argument validation happens before any HIP call
    assert G.conv_loadgen_serve(None, 1, None, None, None, None, None, None, None, None) == cs.CONV_EINVAL
    assert G.conv_loadgen_direct(-1, None, None, None, None, None, 1, None, None, None) == cs.CONV_EINVAL
    g, h = ctypes.c_double(), ctypes.c_double()
    assert G.conv_loadgen_call_latency(4, 1, None, None, None, None, None, None, ctypes.byref(g),
                                       ctypes.byref(h)) == cs.CONV_EINVAL
    assert G.conv_loadgen_call_latency(0, 0, None, None, None, None, None, None, ctypes.byref(g),
                                       ctypes.byref(h)) == cs.CONV_EINVAL
    assert G.conv_loadgen_call_latency(1, 10, None, None, None, None, None, None, ctypes.byref(g),
                                       ctypes.byref(h)) == cs.CONV_EINVAL
    assert G.conv_loadgen_direct(1, None, None, None, None, None, 0, None, None, None) == cs.CONV_EINVAL


def img(planes=3, rows=16, cols=16, dtype=0, pitch=0, plane_stride=0):
    return conv_image(planes, rows, cols, dtype, pitch, plane_stride)


K = (ctypes.c_float * 5)(1, 4, 6, 4, 1)
A, B = 0x100000, 0x900000  # never dereferenced: validation fails first


def call1(i, mode=0, a=A, b=B, k=K):
    return cs.lib().conv_sep5_1pass(ctypes.c_void_p(a), ctypes.c_void_p(b), k,
                                    ctypes.byref(i) if i is not None else None, mode, None)


def call2(i, a=A, b=B, t=0, k=K):
    return cs.lib().conv_sep5_2pass(ctypes.c_void_p(a), ctypes.c_void_p(b), ctypes.c_void_p(t),
                                    k, ctypes.byref(i), None)


@pytest.mark.parametrize("bad", [
    dict(dtype=3), dict(dtype=-1), dict(planes=-1), dict(rows=-2), dict(cols=-5),
    dict(pitch=8), dict(rows=4, plane_stride=10), dict(rows=(1 << 30) + 1),
    dict(cols=(1 << 28) + 1),
    dict(cols=16, pitch=48, plane_stride=15),   # interleaved planes overlapping
    dict(cols=16, pitch=40, plane_stride=16),   # third plane runs past the row
])
def test_1pass_rejects_bad_descriptor(bad):
    assert call1(img(**bad)) == cs.CONV_EINVAL
    assert cs.conv_last_error()


def test_1pass_rejects_null_and_mode():
    assert call1(None) == cs.CONV_EINVAL
    assert call1(img(), k=None) == cs.CONV_EINVAL
    assert call1(img(), mode=2) == cs.CONV_EINVAL
    assert call1(img(), a=0) == cs.CONV_EINVAL
    assert call1(img(), b=0) == cs.CONV_EINVAL


def test_1pass_alias_checks():
    n = 3 * 16 * 16 * 4
    assert call1(img(), a=A, b=A + 4) == cs.CONV_EALIAS
    assert call1(img(), a=A, b=A + n - 4) == cs.CONV_EALIAS
    assert call1(img(), a=A + n - 4, b=A) == cs.CONV_EALIAS


def test_empty_images_are_no_ops():
    # no HIP call happens for an empty image, so this works without a GPU
    for e in (img(planes=0), img(rows=0), img(cols=0)):
        assert call1(e, a=0, b=0) == cs.CONV_OK
        assert call2(e, a=0, b=0) == cs.CONV_OK


def call2x(i, tdt, a=A, b=B, t=0, k=K):
    return cs.lib().conv_sep5_2pass_ex(ctypes.c_void_p(a), ctypes.c_void_p(b), ctypes.c_void_p(t),
                                       k, ctypes.byref(i), tdt, None)


def test_2pass_ex_validation():
    """The 16-bit-intermediate entry point: its own argument checks, all
    before any HIP call."""
    for bad in (-1, 3, 7):
        assert call2x(img(), bad) == cs.CONV_EINVAL
        assert "tmp_dtype" in cs.conv_last_error()
    hwc = img(planes=3, cols=16, pitch=48, plane_stride=1)
    assert call2x(hwc, cs.CONV_F16) == cs.CONV_EINVAL
    assert "FP32 intermediate" in cs.conv_last_error()
    assert call2x(img(), cs.CONV_F16, k=None) == cs.CONV_EINVAL
    assert call2x(img(), cs.CONV_BF16, a=0) == cs.CONV_EINVAL
    assert call2x(img(), cs.CONV_F16, a=A, b=A + 64) == cs.CONV_EALIAS
    # the 16-bit workspace is half the FP32 one: planes*rows*cols*2 bytes
    nt = 3 * 16 * 16 * 2
    assert call2x(img(), cs.CONV_F16, a=A, b=B, t=A - nt + 2) == cs.CONV_EALIAS
    assert call2x(img(), cs.CONV_F16, a=A, b=B, t=B + 3 * 16 * 16 * 4 - 2) == cs.CONV_EALIAS
    for e in (img(planes=0), img(rows=0)):
        assert call2x(e, cs.CONV_F16, a=0, b=0) == cs.CONV_OK


def test_2pass_alias_checks():
    n = 3 * 16 * 16 * 4
    assert call2(img(), a=A, b=A + 64) == cs.CONV_EALIAS          # partial overlap
    assert call2(img(), a=A, b=B, t=A + 8) == cs.CONV_EALIAS     # tmp over input
    assert call2(img(), a=A, b=B, t=B + n - 4) == cs.CONV_EALIAS  # tmp over output
    assert call2(img(pitch=3)) == cs.CONV_EINVAL


def _batch(n, ins, outs, imgs, mode=0, ks=None):
    L = cs.lib()
    pin = (ctypes.c_void_p * max(n, 1))(*ins)
    pout = (ctypes.c_void_p * max(n, 1))(*outs)
    kk = (ctypes.c_float * max(5 * n, 1))(*(ks or [1.0] * (5 * n)))
    ia = (conv_image * max(n, 1))(*imgs)
    return L.conv_sep5_batch(n, pin, pout, kk, ia, mode, None)


def test_batch_validation():
    L = cs.lib()
    assert L.conv_sep5_batch(-1, None, None, None, None, 0, None) == cs.CONV_EINVAL
    assert L.conv_sep5_batch(0, None, None, None, None, 0, None) == cs.CONV_OK
    assert L.conv_sep5_batch(2, None, None, None, None, 0, None) == cs.CONV_EINVAL
    n = 3 * 16 * 16 * 4
    i0 = img()
    # dtype mismatch
    assert _batch(2, [A, A + 2 * n], [B, B + 2 * n], [i0, img(dtype=1)]) == cs.CONV_EINVAL
    # bad mode
    assert _batch(1, [A], [B], [i0], mode=5) == cs.CONV_EINVAL
    # two outputs overlap
    assert _batch(2, [A, A + 2 * n], [B, B + 8], [i0, i0]) == cs.CONV_EALIAS
    # an output overlaps another image's input
    assert _batch(2, [A, B + 2 * n], [B, A + 16], [i0, i0]) == cs.CONV_EALIAS
    # own input/output overlap
    assert _batch(1, [A], [A + 4], [i0]) == cs.CONV_EALIAS
    # a bad descriptor names its image
    assert _batch(2, [A, A + 2 * n], [B, B + 2 * n], [i0, img(rows=-1)]) == cs.CONV_EINVAL
    assert "image 1" in cs.conv_last_error()


def test_tile_cfg_validation_and_roundtrip():
    before = cs.conv_get_tile_cfg(0, 0)
    with pytest.raises(cs.ConvError):
        cs.conv_set_tile_cfg(0, 0, 0, 4)
    with pytest.raises(cs.ConvError):
        cs.conv_set_tile_cfg(0, 0, 32, 3)
    with pytest.raises(cs.ConvError):
        cs.conv_set_tile_cfg(0, 1, 32, 1, 33)
    with pytest.raises(cs.ConvError):
        cs.conv_get_tile_cfg(4, 0)
    b2 = cs.conv_get_tile_cfg(2, 1)
    cs.conv_set_tile_cfg(2, 1, 48, 2, 6, 0, -1)
    c = cs.conv_get_tile_cfg(2, 1)
    assert (c.rows_per_tile, c.waves_per_wg, c.persist_wgs_per_cu, c.pack_tail) == (48, 2, 6, -1)
    cs.conv_set_tile_cfg(2, 1, **b2.as_dict())
    assert cs.conv_get_tile_cfg(2, 1).as_dict() == b2.as_dict()
    assert b2.pack_tail == 0          # default: pack when the launch is large
    with pytest.raises(cs.ConvError):
        cs.conv_set_tile_cfg(0, 0, 8, 1, 0, 4097)   # XCD chunk out of range
    for bad in (-2, 2):
        with pytest.raises(cs.ConvError):
            cs.conv_set_tile_cfg(0, 0, 8, 1, 0, 8, bad)  # pack_tail is -1, 0 or 1
    b16 = cs.conv_get_tile_cfg(1, 0)
    cs.conv_set_tile_cfg(1, 0, 8, 1, 0, 16)
    assert cs.conv_get_tile_cfg(1, 0).xcd_slabs == 16
    cs.conv_set_tile_cfg(1, 0, b16.rows_per_tile, b16.waves_per_wg, 0, b16.xcd_slabs)
    cs.conv_set_tile_cfg(0, 0, before.rows_per_tile, before.waves_per_wg, 0, before.xcd_slabs)
    assert cs.conv_get_tile_cfg(0, 0).as_dict() == before.as_dict()


def test_serve_config_validation():
    L = cs.lib()
    h = ctypes.c_void_p()
    for cfg in (cs.conv_serve_cfg(0, 4, 2, 8, -1, 0, 1), cs.conv_serve_cfg(1 << 30, 0, 2, 8, -1, 0, 1),
                cs.conv_serve_cfg(1 << 30, 4, 0, 8, -1, 0, 1),
                cs.conv_serve_cfg(1 << 30, 4, 17, 8, -1, 0, 1),
                cs.conv_serve_cfg(1 << 30, 4, 2, 0, -1, 0, 1),
                cs.conv_serve_cfg(1 << 30, 4, 2, 8, -1, 0, 2),
                cs.conv_serve_cfg(1 << 30, 4, 2, 8, -1, 0, 1, 2),    # queue_only is 0 or 1
                cs.conv_serve_cfg(1 << 30, 4, 2, 8, -1, 0, 1, 1, -1),  # launch_depth is 0..4
                cs.conv_serve_cfg(1 << 30, 4, 2, 8, -1, 0, 1, 1, 5)):
        assert L.conv_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == cs.CONV_EINVAL
    assert L.conv_serve_poll(None, 1, None) == cs.CONV_EINVAL
    assert L.conv_serve_destroy(None) == cs.CONV_OK


def test_tuner_validation():
    L = cs.lib()
    best = cs.conv_tile_cfg()
    assert L.conv_tune(2, 1, None, None, None, None, 1, None, ctypes.byref(best),
                       None) == cs.CONV_EINVAL
    assert L.conv_tune(0, 0, None, None, None, None, 1, None, ctypes.byref(best),
                       None) == cs.CONV_EINVAL


def test_binding_describes_tensors():
    import torch

    t = torch.zeros(3, 10, 12)
    i = cs.image_of(t)
    assert (i.planes, i.rows, i.cols, i.dtype, i.pitch, i.plane_stride) == (3, 10, 12, 0, 12, 120)
    big = torch.zeros(3, 12, 20, dtype=torch.bfloat16)
    v = big[:, 1:11, 2:14]
    i = cs.image_of(v)
    assert (i.planes, i.rows, i.cols, i.dtype, i.pitch, i.plane_stride) == (3, 10, 12, 2, 20, 240)
    with pytest.raises(TypeError):
        cs.image_of(torch.zeros(2, 2, 2, dtype=torch.float64))


def test_binding_rejects_mismatched_output_layout():
    import torch

    a = torch.zeros(3, 10, 12)
    with pytest.raises(ValueError):
        cs.conv_sep5_1pass(a, torch.zeros(3, 10, 13), [1, 4, 6, 4, 1])
    with pytest.raises(ValueError):
        cs.conv_sep5_2pass(a, torch.zeros(3, 10, 12, dtype=torch.float16), [1, 4, 6, 4, 1])
    big = torch.zeros(3, 10, 16)
    with pytest.raises(ValueError):
        cs.conv_sep5_batch([a], [big[:, :, :12]], [[1, 4, 6, 4, 1]])


def test_row_interleaved_planes_accepted():
    # 3R x C: each row holds the three planes' rows side by side (no GPU call:
    # the empty output pointer check fails after layout validation)
    i = img(planes=3, rows=16, cols=16, pitch=48, plane_stride=16)
    assert call1(i, b=0) == cs.CONV_EINVAL
    assert "NULL" in cs.conv_last_error()


K9 = (ctypes.c_float * 81)(*([1.0] * 81))


def test_width_n_validation():
    L = cs.lib()
    i = img()
    for n in (0, 2, 4, 10, 11, -1):
        assert L.conv_sepn_1pass(A, B, K9, n, ctypes.byref(i), 0, None) == cs.CONV_EINVAL
        assert L.conv_sepn_2pass(A, B, None, K9, n, ctypes.byref(i), None) == cs.CONV_EINVAL
        assert L.conv_2d_direct(A, B, K9, n, ctypes.byref(i), None) == cs.CONV_EINVAL
        assert "width" in cs.conv_last_error()
    assert L.conv_sepn_1pass(A, B, K9, 3, ctypes.byref(i), 2, None) == cs.CONV_EINVAL
    assert L.conv_sepn_1pass(A, B, None, 3, ctypes.byref(i), 0, None) == cs.CONV_EINVAL
    assert L.conv_2d_direct(A, B, None, 3, ctypes.byref(i), None) == cs.CONV_EINVAL
    assert L.conv_2d_direct(0, B, K9, 3, ctypes.byref(i), None) == cs.CONV_EINVAL
    assert L.conv_sepn_1pass(A, A + 4, K9, 7, ctypes.byref(i), 0, None) == cs.CONV_EALIAS
    assert L.conv_2d_direct(A, A + 4, K9, 9, ctypes.byref(i), None) == cs.CONV_EALIAS
    assert L.conv_sepn_2pass(A, B, A + 8, K9, 5, ctypes.byref(i), None) == cs.CONV_EALIAS
    bad = img(pitch=3)
    assert L.conv_2d_direct(A, B, K9, 3, ctypes.byref(bad), None) == cs.CONV_EINVAL
    for e in (img(planes=0), img(rows=0), img(cols=0)):
        for n in (1, 3, 9):
            assert L.conv_sepn_1pass(0, 0, K9, n, ctypes.byref(e), 1, None) == cs.CONV_OK
            assert L.conv_sepn_2pass(0, 0, None, K9, n, ctypes.byref(e), None) == cs.CONV_OK
            assert L.conv_2d_direct(0, 0, K9, n, ctypes.byref(e), None) == cs.CONV_OK


def test_width_n_binding_rejects_non_square_kernel():
    with pytest.raises(ValueError):
        cs._kernel_nn([[1.0, 2.0, 3.0], [4.0, 5.0]])
    taps, n = cs._kernel_nn([[1.0] * 3] * 3)
    assert n == 3 and len(taps) == 9


def test_pyr_down_validation():
    L = cs.lib()
    i = img(planes=3, rows=16, cols=16)
    o = img(planes=3, rows=8, cols=8)
    call = lambda a, ii, b, oo, k=K: L.conv_pyr_down(a, ctypes.byref(ii), b, ctypes.byref(oo), k, None)  # noqa: E731
    assert call(A, i, B, img(planes=3, rows=8, cols=9)) == cs.CONV_EINVAL
    assert call(A, i, B, img(planes=3, rows=7, cols=8)) == cs.CONV_EINVAL
    assert call(A, i, B, img(planes=2, rows=8, cols=8)) == cs.CONV_EINVAL
    assert call(A, i, B, img(planes=3, rows=8, cols=8, dtype=1)) == cs.CONV_EINVAL
    assert call(A, i, B, o, k=None) == cs.CONV_EINVAL
    assert call(0, i, B, o) == cs.CONV_EINVAL
    assert call(A, i, A + 64, o) == cs.CONV_EALIAS
    odd = img(planes=1, rows=7, cols=9)
    assert call(A, odd, B, img(planes=1, rows=4, cols=4)) == cs.CONV_EINVAL
    for e, eo in ((img(rows=0), img(rows=0, cols=8)), (img(cols=0), img(rows=8, cols=0))):
        assert call(0, e, 0, eo) == cs.CONV_OK


def test_hwc_descriptor_validation():
    """plane_stride 1 with 2..4 planes is the pixel-interleaved layout."""
    L = cs.lib()
    ok = img(planes=3, rows=16, cols=16, plane_stride=1)      # pitch 0 -> 48
    assert call1(ok, a=0, b=0) == cs.CONV_EINVAL                # NULL pointers, layout accepted
    assert "NULL" in cs.conv_last_error()
    assert call1(img(planes=5, rows=16, cols=16, plane_stride=1)) == cs.CONV_EINVAL
    assert call1(img(planes=3, rows=16, cols=16, pitch=47, plane_stride=1)) == cs.CONV_EINVAL
    n = 16 * 48 * 4
    assert call1(ok, a=A, b=A + n - 4) == cs.CONV_EALIAS       # extent = rows*cols*planes
    assert call2(ok, a=A, b=B, t=B + 4) == cs.CONV_EALIAS
    # entry points without an HWC kernel refuse it before any HIP call
    pin = (ctypes.c_void_p * 1)(A)
    pout = (ctypes.c_void_p * 1)(B)
    kk = (ctypes.c_float * 5)(1, 1, 1, 1, 1)
    ia = (conv_image * 1)(ok)
    assert L.conv_sep5_batch(1, pin, pout, kk, ia, 0, None) == cs.CONV_EINVAL
    assert "pixel-interleaved" in cs.conv_last_error()
    assert L.conv_sepn_1pass(A, B, K9, 3, ctypes.byref(ok), 0, None) == cs.CONV_EINVAL
    o = img(planes=3, rows=8, cols=8, plane_stride=1)
    assert L.conv_pyr_down(A, ctypes.byref(ok), B, ctypes.byref(o), K, None) == cs.CONV_EINVAL


def test_image_hwc_binding():
    import torch

    t = torch.zeros(5, 7, 3)
    d = cs.image_hwc(t)
    assert (d.planes, d.rows, d.cols, d.pitch, d.plane_stride) == (3, 5, 7, 21, 1)
    with pytest.raises(ValueError):
        cs.image_hwc(torch.zeros(3, 5, 7).permute(1, 0, 2))
    with pytest.raises(ValueError):
        cs.image_of(torch.zeros(5, 7, 3).permute(2, 0, 1))       # columns not contiguous
    with pytest.raises(ValueError):
        cs.image_of(torch.zeros(40).as_strided((3, 5, 7), (1, 7, 1)))


def test_binding_rejects_broadcast_views():
    """Expanded or broadcast tensors repeat memory through a zero stride; the
    descriptor would read 0 as the dense default and cover bytes the tensor
    does not own, so the binding refuses them."""
    import torch

    plane = torch.zeros(1, 16, 24)
    with pytest.raises(ValueError, match="zero stride"):
        cs.image_of(plane.expand(3, 16, 24))
    with pytest.raises(ValueError, match="zero stride"):
        cs.image_of(torch.zeros(3, 1, 24).expand(3, 16, 24))
    with pytest.raises(ValueError, match="zero stride"):
        cs.image_hwc(torch.zeros(16, 24, 1).expand(16, 24, 3))
    # a size-1 dimension may carry any stride, including 0
    d = cs.image_of(plane.expand(1, 16, 24))
    assert (d.planes, d.rows, d.cols) == (1, 16, 24)
    out = torch.zeros(3, 8, 8)
    # the pyramid describes its input without a layout comparison
    with pytest.raises(ValueError, match="zero stride"):
        cs.conv_pyr_down(torch.zeros(1, 16, 16).expand(3, 16, 16), out, [0.2] * 5)


def test_binding_checks_workspace_size():
    """A workspace tensor smaller than planes*rows*cols intermediate values is
    refused before the library would write past it."""
    import torch

    a = torch.zeros(3, 16, 24)
    b = torch.zeros(3, 16, 24)
    k = [0.2] * 5
    with pytest.raises(ValueError, match="workspace"):
        cs.conv_sep5_2pass(a, b, k, d_tmp=torch.empty(3 * 16 * 24 - 1))
    with pytest.raises(ValueError, match="workspace"):
        cs.conv_sep5_2pass(a, b, k, d_tmp=torch.empty(3 * 16 * 24 // 2, dtype=torch.float16))
    with pytest.raises(ValueError, match="workspace"):
        cs.conv_sepn_2pass(a, b, [1.0 / 3] * 3, d_tmp=torch.empty(100))
    with pytest.raises(ValueError, match="workspace"):
        cs.conv_sep5_2pass_ex(a, b, k, cs.CONV_F16,
                              d_tmp=torch.empty(3 * 16 * 24 - 1, dtype=torch.float16))
    with pytest.raises(ValueError, match="contiguous"):
        cs.conv_sep5_2pass(a, b, k, d_tmp=torch.empty(3 * 16 * 24 * 2)[::2])


def test_image_copy_validation():
    L = cs.lib()
    ok = img(planes=3, rows=16, cols=16)
    assert L.conv_image_copy(A, B, None, None) == cs.CONV_EINVAL
    assert L.conv_image_copy(None, B, ctypes.byref(ok), None) == cs.CONV_EINVAL
    assert L.conv_image_copy(A, A + 4, ctypes.byref(ok), None) == cs.CONV_EALIAS
    assert L.conv_image_copy(A, A, ctypes.byref(ok), None) == cs.CONV_OK      # nothing to do
    assert L.conv_image_copy(A, B, ctypes.byref(img(rows=0)), None) == cs.CONV_OK
    assert L.conv_image_copy(A, B, ctypes.byref(img(dtype=7)), None) == cs.CONV_EINVAL


def _tune_entry(**kw):
    e = {"dtype": 0, "kind": 1, "size_class": 3, "rows_per_tile": 16, "waves_per_wg": 2,
         "persist_wgs_per_cu": 4, "xcd_slabs": 1, "pack_tail": 0, "ms": 0.5}
    e.update(kw)
    return e


def test_tuner_cache_roundtrip(tmp_path):
    """The tuner cache file: entries load into their size class only, survive
    a save/load round trip, and an explicit configuration replaces them.
    Host tables only (no GPU)."""
    import json

    d0 = cs.conv_get_tile_cfg(0, 1).as_dict()
    d1 = cs.conv_get_tile_cfg(1, 0).as_dict()
    GiB = 1 << 30
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({"format": "convsep5-tune-1", "arch": "gfx950", "entries": [
        _tune_entry(), _tune_entry(dtype=1, kind=0, size_class=0, rows_per_tile=4,
                                   waves_per_wg=1, persist_wgs_per_cu=0, xcd_slabs=16,
                                   pack_tail=-1, ms=0.01)]}))
    try:
        cs.conv_tune_load(str(p))
        c, tuned = cs.conv_get_tile_cfg_for(0, 1, 2 * GiB)
        assert tuned and (c.rows_per_tile, c.waves_per_wg, c.persist_wgs_per_cu,
                          c.xcd_slabs) == (16, 2, 4, 1)
        c, tuned = cs.conv_get_tile_cfg_for(0, 1, 100 << 20)           # another class
        assert not tuned and c.as_dict() == d0
        c, tuned = cs.conv_get_tile_cfg_for(1, 0, 1 << 20)
        assert tuned and (c.rows_per_tile, c.xcd_slabs, c.pack_tail) == (4, 16, -1)
        assert cs.conv_get_tile_cfg(0, 1).as_dict() == d0               # defaults untouched
        q = tmp_path / "again.json"
        cs.conv_tune_save(str(q))
        saved = json.loads(q.read_text())
        assert saved["format"] == "convsep5-tune-1"
        got = {(e["dtype"], e["kind"], e["size_class"]): e for e in saved["entries"]}
        assert got[(0, 1, 3)]["rows_per_tile"] == 16 and got[(1, 0, 0)]["xcd_slabs"] == 16
        # an explicit configuration drops the tuned entries of its (dtype, kind)
        cs.conv_set_tile_cfg(0, 1, **{k: v for k, v in d0.items()})
        assert not cs.conv_get_tile_cfg_for(0, 1, 2 * GiB)[1]
        assert cs.conv_get_tile_cfg_for(1, 0, 1 << 20)[1]
        cs.conv_tune_load(str(q))
        assert cs.conv_get_tile_cfg_for(0, 1, 2 * GiB)[1]
    finally:
        cs.conv_set_tile_cfg(0, 1, **d0)
        cs.conv_set_tile_cfg(1, 0, **d1)
    assert not cs.conv_get_tile_cfg_for(0, 1, 2 * GiB)[1]
    assert not cs.conv_get_tile_cfg_for(1, 0, 1 << 20)[1]


@pytest.mark.parametrize("bad", [
    {"format": "other", "entries": []},
    {"format": "convsep5-tune-1"},
    {"format": "convsep5-tune-1", "entries": [_tune_entry(rows_per_tile=0)]},
    {"format": "convsep5-tune-1", "entries": [_tune_entry(waves_per_wg=3)]},
    {"format": "convsep5-tune-1", "entries": [_tune_entry(size_class=4)]},
    {"format": "convsep5-tune-1", "entries": [_tune_entry(dtype=3)]},
    {"format": "convsep5-tune-1", "entries": [_tune_entry(), {"dtype": 0}]},
])
def test_tuner_cache_rejects_bad_files(tmp_path, bad):
    import json

    p = tmp_path / "bad.json"
    p.write_text(json.dumps(bad))
    L = cs.lib()
    assert L.conv_tune_load(os.fsencode(str(p))) == cs.CONV_EINVAL
    # all or nothing: the valid first entry of the last case was not installed
    assert not cs.conv_get_tile_cfg_for(0, 1, 2 << 30)[1]
    assert L.conv_tune_load(os.fsencode(str(tmp_path / "missing.json"))) == cs.CONV_ENOTFOUND
    assert L.conv_tune_load(None) == cs.CONV_EINVAL


def test_noalloc_rejects_what_does_not_fit_before_any_hip_call():
    L = cs.lib()
    kk = (ctypes.c_float * 5)(0.1, 0.2, 0.4, 0.2, 0.1)
    dummy_in, dummy_out = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000000000)
    # 3 x 4096 x 4096 FP32 intermediate = 192 MiB > 128 MiB
    big = conv_image(3, 4096, 4096, cs.CONV_F32, 0, 0)
    assert L.conv_sep5_2pass_noalloc(dummy_in, dummy_out, kk, ctypes.byref(big), cs.CONV_F32,
                                     None) == cs.CONV_ENOMEM
    assert "static" in cs.conv_last_error()
    # one byte over, 16-bit intermediate: 2 * planes * rows * cols = 128 MiB + 2
    over = conv_image(1, 1, (cs.CONV_NOALLOC_SCRATCH_BYTES // 2) + 1, cs.CONV_F32, 0, 0)
    assert L.conv_sep5_2pass_noalloc(dummy_in, dummy_out, kk, ctypes.byref(over), cs.CONV_F16,
                                     None) == cs.CONV_ENOMEM
    assert L.conv_sep5_2pass_noalloc(dummy_in, dummy_out, kk, ctypes.byref(big), 7,
                                     None) == cs.CONV_EINVAL
    # nothing to do: no HIP call, no error
    empty = conv_image(3, 0, 4096, cs.CONV_F32, 0, 0)
    assert L.conv_sep5_2pass_noalloc(None, None, kk, ctypes.byref(empty), cs.CONV_F32, None) == cs.CONV_OK


def test_direct_kind_has_its_own_configuration():
    """Kind 2 (the direct 25-tap single-image kernel) is configured apart from
    kind 0: 16-row bands by default for 16-bit storage, 8 for FP32; setting
    one kind leaves the other alone; kind 3 does not exist."""
    assert cs.conv_get_tile_cfg(cs.CONV_F16, cs.KIND_DIRECT).rows_per_tile == 16
    assert cs.conv_get_tile_cfg(cs.CONV_BF16, cs.KIND_DIRECT).rows_per_tile == 16
    assert cs.conv_get_tile_cfg(cs.CONV_F32, cs.KIND_DIRECT).rows_per_tile == 8
    d = cs.conv_get_tile_cfg(cs.CONV_F16, cs.KIND_DIRECT)
    i = cs.conv_get_tile_cfg(cs.CONV_F16, cs.KIND_IMAGE)
    try:
        cs.conv_set_tile_cfg(cs.CONV_F16, cs.KIND_DIRECT, 32, 2, 0, 4)
        assert cs.conv_get_tile_cfg(cs.CONV_F16, cs.KIND_DIRECT).rows_per_tile == 32
        assert cs.conv_get_tile_cfg(cs.CONV_F16, cs.KIND_IMAGE).as_dict() == i.as_dict()
        # a persistent grid applies to the batch kernel only
        cs.conv_set_tile_cfg(cs.CONV_F16, cs.KIND_DIRECT, 16, 1, 8, 8)
        assert cs.conv_get_tile_cfg(cs.CONV_F16, cs.KIND_DIRECT).persist_wgs_per_cu == 0
    finally:
        cs.conv_set_tile_cfg(cs.CONV_F16, cs.KIND_DIRECT, **d.as_dict())
    with pytest.raises(cs.ConvError):
        cs.conv_get_tile_cfg(0, 3)
    with pytest.raises(cs.ConvError):
        cs.conv_set_tile_cfg(0, 3, 8, 1)


def test_tune_cache_holds_direct_kind(tmp_path):
    d = cs.conv_get_tile_cfg(cs.CONV_BF16, cs.KIND_DIRECT).as_dict()
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"format": "convsep5-tune-1", "entries": [
        {"dtype": 2, "kind": 2, "size_class": 1, "rows_per_tile": 32, "waves_per_wg": 1,
         "persist_wgs_per_cu": 0, "xcd_slabs": 8, "pack_tail": 0, "ms": 0.05}]}))
    try:
        cs.conv_tune_load(str(p))
        c, tuned = cs.conv_get_tile_cfg_for(cs.CONV_BF16, cs.KIND_DIRECT, 200 << 20)
        assert tuned and c.rows_per_tile == 32
        assert not cs.conv_get_tile_cfg_for(cs.CONV_BF16, cs.KIND_IMAGE, 200 << 20)[1]
        q = tmp_path / "saved.json"
        cs.conv_tune_save(str(q))
        assert any(e["kind"] == 2 and e["rows_per_tile"] == 32
                   for e in json.loads(q.read_text())["entries"])
    finally:
        cs.conv_set_tile_cfg(cs.CONV_BF16, cs.KIND_DIRECT, **d)
    assert not cs.conv_get_tile_cfg_for(cs.CONV_BF16, cs.KIND_DIRECT, 200 << 20)[1]
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps({"format": "convsep5-tune-1", "entries": [
        {"dtype": 2, "kind": 3, "size_class": 1, "rows_per_tile": 32, "waves_per_wg": 1,
         "persist_wgs_per_cu": 0, "xcd_slabs": 8, "pack_tail": 0, "ms": 0.05}]}))
    with pytest.raises(cs.ConvError):
        cs.conv_tune_load(str(bad))
