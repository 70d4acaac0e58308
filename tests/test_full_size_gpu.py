"""Every pixel of the full-size workloads against the FP64 oracle: one
3 x 4096 x 4096 image and the 64-image batch (H, W = 8*U{30..270}), in FP32
(fused, two-pass and direct 25-tap forms) and stored as FP16 and BF16 (fused),
each in the launch configuration the benchmark times.  FP32 is held to the
1e-6 relative bound; 16-bit storage to the storage gate (the oracle on the
stored input rounded once, or its neighbour at a rounding midpoint).  The
measured maximum relative errors are printed per result, for 16-bit storage
both against the oracle on the stored input and against the oracle on the
FP32 image before it was stored (which adds the input quantisation)."""
import numpy as np
import pytest

import oracle
import paper_1711_09791_amd as cs
from paper_1711_09791_amd import synth
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

LIMIT = {"f16": 2e-3, "bf16": 2.0 ** -8}


def _rel(got64, ref):
    nz = ref != 0
    return float(np.max(np.abs(got64[nz] - ref[nz]) / np.abs(ref[nz]))) if nz.any() else 0.0


def _report(what, **errs):
    print(what + ": " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()), flush=True)


def test_image_fp32_all_forms():
    host = synth.image(1, 3, 4096, 4096)
    k = synth.taps_random(2)
    ref = oracle.conv5(host.astype(np.float64), k.astype(np.float64), nthreads=0)
    a = gu.to_device(host)
    errs = {}
    for form in ("fused", "2pass", "direct"):
        got = gu.to_host_bits(gu.run(form, a, k))
        errs[form] = gu.check_f32(got, ref)
    _report("FP32 3x4096x4096 max rel err", **errs)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_image_16bit(dtype):
    host = synth.image(1, 3, 4096, 4096)
    k = synth.taps_random(2)
    bits = synth.to_storage(host, dtype)
    a = gu.to_device(bits, dtype)
    k64 = k.astype(np.float64)
    ref = oracle.conv5(oracle.decode(bits, dtype), k64, nthreads=0)
    got = gu.to_host_bits(gu.run("fused", a, k))
    e_stored, n_mid = gu.gate16(got, ref, dtype)
    e_fp32 = _rel(oracle.decode(got, dtype), oracle.conv5(host.astype(np.float64), k64, nthreads=0))
    # FP16 within the stated 2e-3; BF16 within its format floor (one rounding)
    assert e_stored <= LIMIT[dtype] * (1 + 1e-6)
    _report(f"{dtype} 3x4096x4096 fused max rel err", vs_stored_input=e_stored,
            vs_fp32_input=e_fp32, midpoint_cases=n_mid)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_batch_64_images(dtype):
    shapes = synth.batch_shapes(3, 64)
    hosts = [synth.image(100 + i, 3, h, w) for i, (h, w) in enumerate(shapes)]
    ks = [synth.taps_random(200 + i) for i in range(64)]
    bits = [synth.to_storage(h, dtype) for h in hosts]
    ins = [gu.to_device(b, dtype) for b in bits]
    outs = [gu.nan_like(a) for a in ins]
    cs.conv_sep5_batch(ins, outs, ks)
    worst, worst_fp32, mids = 0.0, 0.0, 0
    for b, h, o, k in zip(bits, hosts, outs, ks):
        k64 = k.astype(np.float64)
        ref = oracle.conv5(oracle.decode(b, dtype), k64, nthreads=0)
        got = gu.to_host_bits(o)
        if dtype == "f32":
            worst = max(worst, gu.check_f32(got, ref))
        else:
            e, n = gu.gate16(got, ref, dtype)
            worst, mids = max(worst, e), mids + n
            worst_fp32 = max(worst_fp32, _rel(oracle.decode(got, dtype),
                                              oracle.conv5(h.astype(np.float64), k64, nthreads=0)))
    if dtype == "f32":
        _report("FP32 64-image batch max rel err", fused=worst)
    else:
        assert worst <= LIMIT[dtype] * (1 + 1e-6)
        _report(f"{dtype} 64-image batch fused max rel err", vs_stored_input=worst,
                vs_fp32_input=worst_fp32, midpoint_cases=mids)
