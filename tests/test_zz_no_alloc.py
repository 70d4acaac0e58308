"""The allocation-free two-pass entry point, conv_sep5_2pass_noalloc, called
through the C ABI, against conv_sep5_2pass_ex with a caller's workspace (the
same kernels, so the bar is bitwise equality): two calls in a row, the
second on a smaller image, so that the static workspace holds the first
call's values when the second runs; every storage type and intermediate type;
in place; on a stream of its own; and the FP32 result against the FP64 oracle.
"""
import ctypes

import numpy as np
import pytest

import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TDT = {"f32": cs.CONV_F32, "f16": cs.CONV_F16, "bf16": cs.CONV_BF16}
# the first call larger than the second; ragged widths and heights
SHAPES = [(3, 1031, 2085), (3, 260, 333)]


def _torch():
    import torch

    return torch


def _device_image(seed, shape, dtype):
    torch = _torch()
    a = torch.from_numpy(synth.image(seed, *shape)).cuda()
    return a.to(getattr(torch, gu.TORCH_DT[dtype]))


def _noalloc(a, o, k, tdt, stream=None):
    """One call of the entry point through the C ABI (arguments marshalled by hand)."""
    torch = _torch()
    img = cs.image_of(a)
    kk = (ctypes.c_float * 5)(*[float(v) for v in k])
    s = (stream or torch.cuda.current_stream()).cuda_stream
    return cs.lib().conv_sep5_2pass_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(o.data_ptr()),
                                            kk, ctypes.byref(img), int(tdt), ctypes.c_void_p(s))


def _with_workspace(a, o, k, tdt):
    torch = _torch()
    n = a.numel()
    ws = torch.empty(n, dtype=torch.float32 if tdt == cs.CONV_F32 else torch.float16, device=a.device)
    cs.conv_sep5_2pass_ex(a, o, k, tdt, d_tmp=ws)


def _bits(t):
    torch = _torch()
    t = t.detach().contiguous()
    return t.view(torch.int32) if t.element_size() == 4 else t.view(torch.int16)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("tname", ["f32", "f16", "bf16"])
def test_two_calls_in_a_row_equal_the_workspace_form(dtype, tname):
    torch = _torch()
    tdt = TDT[tname]
    k = synth.taps_random(77)
    for i, shape in enumerate(SHAPES):
        print(f"noalloc: storage {dtype}, intermediate {tname}, shape {shape}", flush=True)
        a = _device_image(600 + i, shape, dtype)
        ref, got = gu.nan_like(a), gu.nan_like(a)
        _with_workspace(a, ref, k, tdt)
        st = _noalloc(a, got, k, tdt)
        assert st == cs.CONV_OK, cs.conv_last_error()
        torch.cuda.synchronize()
        assert torch.equal(_bits(got), _bits(ref)), (dtype, tname, shape)


def test_fp32_matches_the_oracle():
    torch = _torch()
    k = synth.taps_random(78)
    for i, shape in enumerate(SHAPES):
        host = synth.image(610 + i, *shape)
        a = gu.to_device(host)
        out = gu.nan_like(a)
        assert _noalloc(a, out, k, cs.CONV_F32) == cs.CONV_OK, cs.conv_last_error()
        torch.cuda.synchronize()
        gu.check_f32(out.cpu().numpy(), gu.oracle_of(host, k))


def test_in_place_and_own_stream():
    torch = _torch()
    k = synth.taps_random(79)
    s = torch.cuda.Stream()
    for i, shape in enumerate(SHAPES):
        a = _device_image(620 + i, shape, "f32")
        ref = gu.nan_like(a)
        _with_workspace(a, ref, k, cs.CONV_F32)
        b = a.clone()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            assert _noalloc(b, b, k, cs.CONV_F32, stream=s) == cs.CONV_OK, cs.conv_last_error()
        s.synchronize()
        assert torch.equal(_bits(b), _bits(ref)), shape


def test_largest_fitting_intermediate():
    """3 x 3840 x 2160 FP32: 99.5 MB of FP32 intermediate, within the 128 MiB workspace."""
    torch = _torch()
    k = synth.taps_random(80)
    a = torch.rand(3, 2160, 3840, device="cuda")
    ref, got = gu.nan_like(a), gu.nan_like(a)
    _with_workspace(a, ref, k, cs.CONV_F32)
    assert _noalloc(a, got, k, cs.CONV_F32) == cs.CONV_OK, cs.conv_last_error()
    torch.cuda.synchronize()
    assert torch.equal(_bits(got), _bits(ref))


def test_takes_no_device_memory():
    """Twenty calls on a 3 x 2048 x 2048 image (48 MiB of FP32 intermediate)
    leave the device's free memory exactly as it was (hipMemGetInfo, read
    through torch): no allocation, not even a stream-ordered one."""
    torch = _torch()
    k = synth.taps_random(81)
    a = torch.rand(3, 2048, 2048, device="cuda")
    out = torch.empty_like(a)
    assert _noalloc(a, out, k, cs.CONV_F32) == cs.CONV_OK, cs.conv_last_error()  # first use on the device
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(20):
        assert _noalloc(a, out, k, cs.CONV_F32) == cs.CONV_OK, cs.conv_last_error()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
