#!/usr/bin/env python3
"""Throughput of the width-5 separable convolution on one MI355X.

Headline workload: one 3-plane 4096 x 4096 FP32 image (uniform [0,1) pixels,
seed 1), positive random taps normalised to sum 1 (seed 2); 2-pixel border 0.
A step is one fused single-pass convolution of the image (input read, row
filter, on-chip intermediate, column filter, border, output store); `value` is
its MPix/s.  Inputs are resident in HBM; timed launches rotate over several
input/output buffer sets so the working set exceeds the 256 MB Infinity Cache.

Also measured (the headline line carries a compact summary; every figure goes
to --detail-out, or to one stderr line):
  forms      the two-pass form (HBM intermediate), the two-pass form with a
             16-bit intermediate, the direct 25-tap form, the copy-back single
             pass, the in-place two-pass, the library's own image copy of the
             same bytes (the achievable ceiling) and torch's copy; every form
             also against the problem's minimum of 8 B per plane-pixel; the
             fused form also cache-warm (one buffer set);
  small      3x256x256: microseconds per call of each form, cold and warm,
             queued and as a lone round trip, beside an empty kernel's launch;
  precision  the image stored as FP16 and BF16 (FP32 accumulation);
  batch      64 uneven images (H, W = 8*U{30..270}) in one launch (FP32,
             and the same images stored as FP16 and BF16), eager (FP32 also
             as a captured graph), with the default and the autotuned tile
             configuration, against one launch per image;
  serving    Poisson arrivals of 640x480 .. 3840x2160 frames, each with its
             own taps: p50/p99 latency (from each request's scheduled
             arrival to its completion) of the continuous-batching server
             against one launch per request (1 or 4 streams), at 0.5x and
             0.8x of the batched server's measured capacity, median of three
             interleaved repetitions; and 640x480 only;
  widths     odd widths n = 1..9 on the same image: fused, two-pass and
             direct (n*n terms) separable forms and a full non-separable
             n x n kernel, each against the HBM and the FP32 ALU roofline
             (the O(n) vs O(n^2) trade-off of Section 5.1);
  hwc        the same image stored pixel-interleaved (packed RGB);
  pyramid    one blur + 2x decimation level of the same image (FP32, FP16);
  cpu_baseline  the FP64 oracle on the host cores (all, and one) on the image
             and on the 64-image batch.

Prints ONE JSON line on stdout.  Run with no flags for the default configuration.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

P, R, C = 3, 4096, 4096
HBM_PEAK_GBS = 8000.0
# FP32 vector FMA rate without packed FP32 math (the kernels are built with
# packed FP32 off): 256 CUs x 64 lanes x 2 flop x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
SETTLE_S = 0.03  # seconds of untimed launches before each image's first form
KERNEL_DIR = os.path.join(ROOT, "paper_1711_09791_amd", "csrc")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    # After an idle moment the GPU's clocks dip and recover over ~600 launches
    # (~25 ms) of this kernel; 1000 warm-up launches reach the steady state.
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--sets", type=int, default=3, help="rotating buffer sets")
    ap.add_argument("--forms", default="fused,2pass,direct25,copy,torch_copy,1pass_copyback,"
                                       "2pass_inplace,2pass_t16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision, widths, batch and serving measurements")
    ap.add_argument("--extras", default="small,precision,widths,hwc,pyramid,batch,serving",
                    help="comma list of extra measurements to run")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the cache-warm timing of the fused form on one buffer set")
    ap.add_argument("--detail-out", default=None,
                    help="write every figure as JSON to this file (default: one line on stderr)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-reps", type=int, default=3,
                    help="repetitions of each serving point (medians reported)")
    ap.add_argument("--cpu-min-s", type=float, default=10.0,
                    help="repeat the oracle until this much CPU time is spent")
    return ap.parse_args()


# the sources the width-5 kernels (whose traffic profiles/traffic.json records)
# are compiled from
TRAFFIC_SOURCES = ("conv_internal.h", "conv_kernels.h", "conv_kernels_bf16.hip", "conv_kernels_f16.hip",
                   "conv_kernels_f32.hip")


def kernel_src_sha() -> str:
    """sha256 over the sources of the width-5 kernels (TRAFFIC_SOURCES)."""
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(KERNEL_DIR, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def traffic_for(form: str):
    """HBM bytes per launch measured by rocprofv3 counters, if they were taken
    on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha256") != kernel_src_sha():
        return None
    e = t.get("workloads", {}).get(form)
    return None if e is None else e.get("bytes_per_launch")


def timed(torch, fn, steps, warmup):
    """ms over `steps` back-to-back calls, from a pair of HIP events recorded
    on torch's current stream (the stream every call here launches on) around
    the whole timed region, bracketed by device synchronisation.  No event
    sits between the launches, so total / steps is the average launch
    duration including only the GPU's own gap between consecutive kernels."""
    for i in range(warmup):
        fn(i)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for i in range(steps):
        fn(i)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


_T0 = time.perf_counter()


def progress(msg: str) -> None:
    """One line on stderr per finished measurement (the JSON line is stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def check(cs, st):
    if st != 0:
        raise cs.ConvError(st, cs.conv_last_error())


def bench_image(torch, cs, host, k, args, dtype=None, forms=("fused", "2pass", "direct25", "copy")):
    """One 3x4096x4096 image, rotating buffer sets; returns per-form figures."""
    dev = torch.device("cuda:0")
    base = torch.from_numpy(host).to(dev)
    if dtype is not None:
        base = base.to(dtype)
    esz = base.element_size()
    S = max(1, args.sets)
    ins = [base] + [base.clone() for _ in range(S - 1)]
    outs = [torch.empty_like(base) for _ in range(S)]
    tmp = torch.empty(P * R * C, device=dev) if any(f.startswith("2pass") for f in forms) else None
    # the 16-bit intermediate: FP16 for FP32 and FP16 images, BF16 for BF16 images
    t16 = cs.CONV_BF16 if base.dtype == torch.bfloat16 else cs.CONV_F16
    for o in outs:  # the in-place forms work on the output buffers
        o.copy_(base)
    L = cs.lib()
    img = cs.image_of(base)
    kk = (ctypes.c_float * 5)(*[float(v) for v in k])
    hs = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pin = [ctypes.c_void_p(t.data_ptr()) for t in ins]
    pout = [ctypes.c_void_p(t.data_ptr()) for t in outs]
    ptmp = ctypes.c_void_p(tmp.data_ptr()) if tmp is not None else None
    pimg = ctypes.byref(img)
    steps_fn = {
        # the paper's in-place variants (Section 7): copy-back single-pass, in-place two-pass
        "1pass_copyback": lambda i: check(cs, L.conv_sep5_1pass(pout[i % S], pout[i % S], kk, pimg, 0, hs)),
        "2pass_inplace": lambda i: check(cs, L.conv_sep5_2pass(pout[i % S], pout[i % S], ptmp, kk, pimg, hs)),
        "fused": lambda i: check(cs, L.conv_sep5_1pass(pin[i % S], pout[i % S], kk, pimg, 0, hs)),
        "direct25": lambda i: check(cs, L.conv_sep5_1pass(pin[i % S], pout[i % S], kk, pimg, 1, hs)),
        "2pass": lambda i: check(cs, L.conv_sep5_2pass(pin[i % S], pout[i % S], ptmp, kk, pimg, hs)),
        "2pass_t16": lambda i: check(cs, L.conv_sep5_2pass_ex(pin[i % S], pout[i % S], ptmp, kk, pimg,
                                                              t16, hs)),
        # the library's own streaming copy of the same bytes: the achievable ceiling
        "copy": lambda i: check(cs, L.conv_image_copy(pin[i % S], pout[i % S], pimg, hs)),
        "torch_copy": lambda i: outs[i % S].copy_(ins[i % S]),
    }
    # bytes each form moves by its own definition (the two-pass forms count
    # their intermediate, written and read back) ...
    alg_bytes = {"fused": 2 * esz, "direct25": 2 * esz, "2pass": 2 * esz + 8, "copy": 2 * esz,
                 "torch_copy": 2 * esz, "1pass_copyback": 4 * esz, "2pass_inplace": 2 * esz + 8,
                 "2pass_t16": 2 * esz + 4}
    # ... and the problem's minimum: read the image once, write the result once
    min_bytes = 2 * esz * P * R * C
    launches = {"2pass": 2, "2pass_inplace": 2, "1pass_copyback": 2, "2pass_t16": 2}
    res = {}
    # Clock settle (untimed, outside the warm-up count): after an idle moment the
    # GPU's clocks take ~25 ms of these launches to recover, so the first form
    # runs for SETTLE_S of wall time before its warm-up steps whatever --warmup is.
    if forms:
        fn0 = steps_fn[forms[0]]
        torch.cuda.synchronize()
        t_end = time.perf_counter() + SETTLE_S
        i = 0
        while time.perf_counter() < t_end:
            fn0(i)
            i += 1
            if i % 64 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
    for name in forms:
        total = timed(torch, steps_fn[name], args.steps, args.warmup)
        avg = total / args.steps
        nbytes = alg_bytes[name] * P * R * C
        res[name] = {
            "ms_per_step": avg,
            "avg_launch_ms": avg / launches.get(name, 1),
            "launches_per_step": launches.get(name, 1),
            "mpix_per_s": (R * C) / (avg * 1e-3) / 1e6,
            "alg_bytes_per_step": nbytes,
            "alg_GBps": nbytes / (avg * 1e-3) / 1e9,
            # against the problem's minimum bytes: comparable across forms
            "frac_of_hbm_peak": min_bytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
        if nbytes != min_bytes:
            # the form's own bytes over the time; for the two-pass forms most of
            # the intermediate is read back from the Infinity Cache, so this is
            # a memory-system rate, not an HBM-only one
            res[name]["own_bytes_frac_of_peak"] = nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS
    if "fused" in res and not getattr(args, "no_warm", False):
        # warm: the same input and output every launch (402 MB for FP32, of which
        # the 256 MB Infinity Cache keeps part); cold: the rotating sets above
        fn = lambda i: check(cs, L.conv_sep5_1pass(pin[0], pout[0], kk, pimg, 0, hs))  # noqa: E731
        res["fused"]["warm_same_buffers_avg_launch_ms"] = timed(torch, fn, args.steps, args.warmup) / args.steps
    for c in ("copy", "torch_copy"):
        if "fused" in res and c in res:
            res["fused"]["frac_of_" + c] = res[c]["avg_launch_ms"] / res["fused"]["avg_launch_ms"]
    eq = None
    if "fused" in res and "2pass" in res:
        o1, o2 = torch.empty_like(base), torch.empty_like(base)
        cs.conv_sep5_1pass(base, o1, k)
        cs.conv_sep5_2pass(base, o2, k, d_tmp=tmp)
        torch.cuda.synchronize()
        eq = bool(torch.equal(o1, o2))
    del ins, outs, tmp
    return res, eq


def bench_small(torch, cs, synth, args):
    """The small configuration (3x256x256 FP32, seed 0, taps [1,4,6,4,1]/16):
    microseconds per call of each form, next to a launch of an empty kernel
    (the GPU's fixed cost per call, as the paper's empty tasks and kernels
    measure the runtimes' overhead, Section 6 Table 2); compute = call - empty.
    gpu_us: calls queued back to back (events around n calls), warm (one
    buffer set, 1.5 MB, held in cache) and cold (256 rotating sets, 403 MB,
    more than the 256 MB Infinity Cache).  host_us: median submit-to-done
    latency of a lone call (launch + stream synchronisation), native clock."""
    G = cs.loadgen_lib()
    L = cs.lib()
    Ps, Rs, Cs = 3, 256, 256
    host = synth.image(0, Ps, Rs, Cs)
    k = synth.taps_binomial()
    base = torch.from_numpy(host).cuda()
    out = torch.empty_like(base)
    tmp = torch.empty(Ps * Rs * Cs, device="cuda")
    img = cs.image_of(base)
    kk = (ctypes.c_float * 5)(*[float(v) for v in k])
    hs = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n = 2000
    res = {}
    for form, name in ((0, "empty_kernel"), (1, "fused"), (2, "direct25"), (3, "2pass")):
        g, h = ctypes.c_double(), ctypes.c_double()
        check(cs, G.conv_loadgen_call_latency(form, n, base.data_ptr(), out.data_ptr(), tmp.data_ptr(),
                                              kk, ctypes.byref(img), hs, ctypes.byref(g),
                                              ctypes.byref(h)))
        res[name] = {"gpu_us_warm": g.value, "host_us": h.value}
    # cold: rotate over enough buffer sets that no launch finds its bytes in a cache
    NS = 256
    ins = [base.clone() for _ in range(NS)]
    outs = [torch.empty_like(base) for _ in range(NS)]
    tmps = [torch.empty(Ps * Rs * Cs, device="cuda") for _ in range(NS)]
    pin = [ctypes.c_void_p(t.data_ptr()) for t in ins]
    pout = [ctypes.c_void_p(t.data_ptr()) for t in outs]
    ptmp = [ctypes.c_void_p(t.data_ptr()) for t in tmps]
    pimg = ctypes.byref(img)
    fns = {
        "fused": lambda i: check(cs, L.conv_sep5_1pass(pin[i % NS], pout[i % NS], kk, pimg, 0, hs)),
        "direct25": lambda i: check(cs, L.conv_sep5_1pass(pin[i % NS], pout[i % NS], kk, pimg, 1, hs)),
        "2pass": lambda i: check(cs, L.conv_sep5_2pass(pin[i % NS], pout[i % NS], ptmp[i % NS], kk,
                                                       pimg, hs)),
    }
    for name, fn in fns.items():
        res[name]["gpu_us_cold"] = 1e3 * timed(torch, fn, 4 * NS, NS) / (4 * NS)
    e = res["empty_kernel"]
    for name in fns:
        r = res[name]
        r["compute_gpu_us_warm"] = r["gpu_us_warm"] - e["gpu_us_warm"]
        r["compute_host_us"] = r["host_us"] - e["host_us"]
    del ins, outs, tmps
    return {"workload": f"3x{Rs}x{Cs} FP32, seed 0, k=[1,4,6,4,1]/16", "calls": n, "results": res}


def bench_widths(torch, cs, synth, host, args, widths=(1, 3, 5, 7, 9)):
    """Width-n forms on the 3x4096x4096 FP32 image: time per launch, MPix/s and
    both rooflines.  flops per plane-pixel: an n-tap filter is 1 multiply and
    n-1 FMAs (2n-1 flops); fused / two-pass run two of them, the direct forms n
    row chains plus n-1 adds (2n^2-1).  The full n x n kernel at n = 7, 9 is
    also timed on the same image in FP16 storage."""
    dev = torch.device("cuda:0")
    base = torch.from_numpy(host).to(dev)
    S = max(1, args.sets)
    ins = [base] + [base.clone() for _ in range(S - 1)]
    outs = [torch.empty_like(base) for _ in range(S)]
    tmp = torch.empty(P * R * C, device=dev)
    L = cs.lib()
    img = cs.image_of(base)
    pimg = ctypes.byref(img)
    hs = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pin = [ctypes.c_void_p(t.data_ptr()) for t in ins]
    pout = [ctypes.c_void_p(t.data_ptr()) for t in outs]
    ptmp = ctypes.c_void_p(tmp.data_ptr())
    steps = max(10, min(args.steps, 100))
    res = {}
    for n in widths:
        k = synth.taps_random_n(2 + n, n)
        K = synth.kernel_signed(3 + n, n)
        kk = (ctypes.c_float * n)(*[float(v) for v in k])
        KK = (ctypes.c_float * (n * n))(*[float(v) for v in K.reshape(-1)])
        fns = {
            "fused": lambda i: check(cs, L.conv_sepn_1pass(pin[i % S], pout[i % S], kk, n, pimg, 0, hs)),
            "2pass": lambda i: check(cs, L.conv_sepn_2pass(pin[i % S], pout[i % S], ptmp, kk, n, pimg, hs)),
            "direct": lambda i: check(cs, L.conv_sepn_1pass(pin[i % S], pout[i % S], kk, n, pimg, 1, hs)),
            "full": lambda i: check(cs, L.conv_2d_direct(pin[i % S], pout[i % S], KK, n, pimg, hs)),
        }
        row = {}
        for name, fn in fns.items():
            avg = timed(torch, fn, steps, max(3, args.warmup // 2)) / steps
            nbytes = (16 if name == "2pass" else 8) * P * R * C
            flops = ((4 * n - 2) if name in ("fused", "2pass") else (2 * n * n - 1)) * P * R * C
            row[name] = {
                "ms_per_step": avg,
                "mpix_per_s": (R * C) / (avg * 1e-3) / 1e6,
                "frac_of_hbm_peak": nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "frac_of_alu_peak": flops / (avg * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
            }
        res[f"n{n}"] = row
    del ins, outs, tmp
    # the direct n x n forms on FP16 storage (4 B per plane-pixel), n = 7, 9
    ins16 = [base.half()] + [base.half() for _ in range(S - 1)]
    outs16 = [torch.empty_like(ins16[0]) for _ in range(S)]
    img16 = cs.image_of(ins16[0])
    p16 = ctypes.byref(img16)
    pin16 = [ctypes.c_void_p(t.data_ptr()) for t in ins16]
    pout16 = [ctypes.c_void_p(t.data_ptr()) for t in outs16]
    res16 = {}
    for n in (7, 9):
        K = synth.kernel_signed(3 + n, n)
        KK = (ctypes.c_float * (n * n))(*[float(v) for v in K.reshape(-1)])
        fn = lambda i: check(cs, L.conv_2d_direct(pin16[i % S], pout16[i % S], KK, n, p16, hs))  # noqa: E731
        avg = timed(torch, fn, steps, max(3, args.warmup // 2)) / steps
        res16[f"n{n}"] = {"full": {
            "ms_per_step": avg,
            "mpix_per_s": (R * C) / (avg * 1e-3) / 1e6,
            "frac_of_hbm_peak": 4 * P * R * C / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "frac_of_alu_peak": (2 * n * n - 1) * P * R * C / (avg * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
        }}
    del ins16, outs16
    return {"alu_peak_tflops": ALU_PEAK_TFLOPS, "steps": steps, "results": res, "f16_results": res16}


def bench_hwc(torch, cs, host, k, args):
    """The 3x4096x4096 FP32 image as packed RGB ([rows, cols, 3]): fused,
    direct and two-pass forms (same bytes as the planar forms)."""
    S = max(1, args.sets)
    base = torch.from_numpy(host).cuda().permute(1, 2, 0).contiguous()
    ins = [base] + [base.clone() for _ in range(S - 1)]
    outs = [torch.empty_like(base) for _ in range(S)]
    tmp = torch.empty(P * R * C, device="cuda")
    L = cs.lib()
    img = cs.image_hwc(base)
    kk = (ctypes.c_float * 5)(*[float(v) for v in k])
    hs = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pin = [ctypes.c_void_p(t.data_ptr()) for t in ins]
    pout = [ctypes.c_void_p(t.data_ptr()) for t in outs]
    ptmp = ctypes.c_void_p(tmp.data_ptr())
    fns = {
        "fused": lambda i: check(cs, L.conv_sep5_1pass(pin[i % S], pout[i % S], kk, ctypes.byref(img), 0, hs)),
        "direct25": lambda i: check(cs, L.conv_sep5_1pass(pin[i % S], pout[i % S], kk, ctypes.byref(img), 1, hs)),
        "2pass": lambda i: check(cs, L.conv_sep5_2pass(pin[i % S], pout[i % S], ptmp, kk, ctypes.byref(img), hs)),
    }
    res = {}
    for name, fn in fns.items():
        avg = timed(torch, fn, args.steps, args.warmup) / args.steps
        nbytes = (16 if name == "2pass" else 8) * P * R * C
        res[name] = {
            "ms_per_step": avg,
            "mpix_per_s": (R * C) / (avg * 1e-3) / 1e6,
            "alg_GBps": nbytes / (avg * 1e-3) / 1e9,
            "frac_of_hbm_peak": nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
    del ins, outs, tmp, base
    return res


def bench_pyramid(torch, cs, host, k, args):
    """conv_pyr_down on the 3x4096x4096 image in FP32 and FP16 storage."""
    res = {}
    S = max(1, args.sets)
    L = cs.lib()
    kk = (ctypes.c_float * 5)(*[float(v) for v in k])
    hs = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for name, dt in (("f32", torch.float32), ("f16", torch.float16)):
        base = torch.from_numpy(host).cuda().to(dt)
        ins = [base] + [base.clone() for _ in range(S - 1)]
        outs = [torch.empty(P, (R + 1) // 2, (C + 1) // 2, dtype=dt, device="cuda") for _ in range(S)]
        ii, oi = cs.image_of(base), cs.image_of(outs[0])
        pin = [ctypes.c_void_p(t.data_ptr()) for t in ins]
        pout = [ctypes.c_void_p(t.data_ptr()) for t in outs]
        fn = lambda i: check(cs, L.conv_pyr_down(pin[i % S], ctypes.byref(ii), pout[i % S],  # noqa: E731
                                                 ctypes.byref(oi), kk, hs))
        avg = timed(torch, fn, args.steps, args.warmup) / args.steps
        esz = base.element_size()
        nbytes = esz * P * R * C + esz * P * ((R + 1) // 2) * ((C + 1) // 2)
        res[name] = {
            "ms_per_step": avg,
            "input_mpix_per_s": (R * C) / (avg * 1e-3) / 1e6,
            "alg_bytes_per_step": nbytes,
            "alg_GBps": nbytes / (avg * 1e-3) / 1e9,
            "frac_of_hbm_peak": nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
        del ins, outs, base
    return res


def bench_batch(torch, cs, synth, args):
    """64 uneven images: persistent batch launch, graph replay (FP32), one
    launch per image; FP32, then the same batch stored as FP16 and BF16."""
    shapes = synth.batch_shapes(3, 64)
    pix = sum(h * w for h, w in shapes)
    steps = max(20, args.steps // 4)
    warm = max(3, args.warmup // 10)
    ks = [synth.taps_random(200 + i) for i in range(64)]
    res = {}
    for dt, tdt, esz in (("f32", torch.float32, 4), ("f16", torch.float16, 2),
                         ("bf16", torch.bfloat16, 2)):
        ins = [torch.from_numpy(synth.image(100 + i, 3, h, w)).cuda().to(tdt)
               for i, (h, w) in enumerate(shapes)]
        outs = [torch.empty_like(a) for a in ins]
        nbytes = 6 * esz * pix
        # arguments marshalled once, so that the timed loops measure the launches
        L = cs.lib()
        n = len(ins)
        pin = (ctypes.c_void_p * n)(*[a.data_ptr() for a in ins])
        pout = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        kk = (ctypes.c_float * (5 * n))(*[float(v) for k in ks for v in k])
        imgs = (cs.conv_image * n)(*[cs.image_of(a) for a in ins])
        hs = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        t_eager = timed(torch, lambda i: check(cs, L.conv_sep5_batch(n, pin, pout, kk, imgs, 0, hs)),
                        steps, warm)
        t_graph = None
        if dt == "f32":
            plan = cs.conv_batch_plan_create(ins, outs, ks)
            t_graph = timed(torch, lambda i: plan.launch(), steps, warm)
            plan.destroy()
        one = [(ctypes.c_void_p(pin[j]), ctypes.c_void_p(pout[j]),
                (ctypes.c_float * 5)(*kk[5 * j:5 * j + 5]), ctypes.byref(imgs[j])) for j in range(n)]

        def lone(i):
            for a, o, k, im in one:
                check(cs, L.conv_sep5_1pass(a, o, k, im, 0, hs))

        t_lone = timed(torch, lone, steps, warm)
        # the autotuner on this batch (kind 1): installs its choice for the
        # batch's storage type and size class; the eager launch is timed again
        # with it, then the default is restored
        dcode = {"f32": 0, "f16": 1, "bf16": 2}[dt]
        default_cfg = cs.conv_get_tile_cfg(dcode, 1)
        tuned_cfg, _ = cs.conv_tune(1, ins, outs, ks, reps=5)
        t_tuned = timed(torch, lambda i: check(cs, L.conv_sep5_batch(n, pin, pout, kk, imgs, 0, hs)),
                        steps, warm)
        cs.conv_set_tile_cfg(dcode, 1, **default_cfg.as_dict())
        ms_e, ms_l = t_eager / steps, t_lone / steps
        r = {
            "images": 64, "mpix": pix / 1e6, "alg_bytes": nbytes,
            "tile_cfg": cs.conv_get_tile_cfg({"f32": 0, "f16": 1, "bf16": 2}[dt], 1).as_dict(),
            "eager_ms": ms_e, "per_image_launches_ms": ms_l,
            "eager_mpix_per_s": pix / (ms_e * 1e-3) / 1e6,
            "per_image_mpix_per_s": pix / (ms_l * 1e-3) / 1e6,
            "eager_alg_GBps": nbytes / (ms_e * 1e-3) / 1e9,
            "eager_frac_of_hbm_peak": nbytes / (ms_e * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "speedup_vs_per_image": ms_l / ms_e,
            "tuned_cfg": tuned_cfg.as_dict(),
            "tuned_eager_ms": t_tuned / steps,
            "tuned_eager_frac_of_hbm_peak": nbytes / (t_tuned / steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
        if t_graph is not None:
            ms_g = t_graph / steps
            r.update({
                "graph_ms": ms_g,
                "graph_mpix_per_s": pix / (ms_g * 1e-3) / 1e6,
                "graph_alg_GBps": nbytes / (ms_g * 1e-3) / 1e9,
                "graph_frac_of_hbm_peak": nbytes / (ms_g * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "speedup_vs_per_image": ms_l / ms_g,
            })
        res[dt] = r
        del ins, outs
    out = dict(res["f32"])
    out["16bit"] = {"f16": res["f16"], "bf16": res["bf16"]}
    return out


def bench_serving(torch, cs, synth, args, sizes=None):
    """Poisson request stream (arrival times kept by the native load generator);
    continuous batching vs one conv_sep5_1pass launch per request."""
    G = cs.loadgen_lib()
    sizes = list(sizes or synth.SERVE_SIZES)
    NBUF = 64  # >= max_slots: two requests admitted together never share a buffer
    bufs = {}
    for (h, w) in sizes:
        ins = [torch.rand(3, h, w, device="cuda") for _ in range(NBUF)]
        outs = [torch.empty_like(ins[0]) for _ in range(NBUF)]
        bufs[(h, w)] = (ins, outs, cs.image_of(ins[0]))
    torch.cuda.synchronize()
    hs = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    budget = 8 << 30

    def requests(n, rate, seed):
        arrivals, req_sizes = synth.serving_stream(seed, seed + 1, n, rate if rate else 1.0, sizes)
        if not rate:
            arrivals = arrivals * 0.0  # everything at once: capacity probe
        arr = (ctypes.c_double * n)(*[float(a) for a in arrivals])
        pin, pout = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
        imgs = (cs.conv_image * n)()
        flat = []
        counters = {s: 0 for s in sizes}
        for i, s in enumerate(req_sizes):
            ins, outs, img = bufs[s]
            j = counters[s] % NBUF
            counters[s] += 1
            pin[i], pout[i], imgs[i] = ins[j].data_ptr(), outs[j].data_ptr(), img
            flat.extend(float(v) for v in synth.taps_random(6000 + i))
        kk = (ctypes.c_float * (5 * n))(*flat)
        return arr, pin, pout, kk, imgs

    q = lambda v, p: v[min(len(v) - 1, int(p * len(v)))]  # noqa: E731

    def summarize(sub, done, lag, n, warm, rate, extra):
        # latency from the request's scheduled arrival: the time from submit to
        # done plus how late the load generator submitted it (a submitting
        # thread that is still busy launching the previous request delays the
        # next one; that wait belongs to the request's latency)
        lat = sorted((d - s) / 1e3 + lg * 1e6 for s, d, lg in zip(sub[warm:], done[warm:], lag[warm:]))
        lat_sub = sorted((d - s) / 1e3 for s, d in zip(sub[warm:], done[warm:]))
        span = (max(done[warm:]) - min(sub[warm:])) / 1e9
        lg = sorted(lag)
        return {"p50_us": q(lat, 0.50), "p99_us": q(lat, 0.99), "mean_us": sum(lat) / len(lat),
                "p50_from_submit_us": q(lat_sub, 0.50), "p99_from_submit_us": q(lat_sub, 0.99),
                "throughput_req_per_s": (n - warm) / span, "offered_req_per_s": rate,
                "submit_lag_p99_us": q(lg, 0.99) * 1e6, **extra}

    def run_server(max_batch, n_streams, max_bytes, rate, n, warm, seed=5, queue_only=False, depth=1):
        arr, pin, pout, kk, imgs = requests(n, rate, seed)
        # inputs are static and synchronised: no producer ordering, like the
        # direct-launch baseline
        srv = cs.Server(budget, max_slots=NBUF, n_streams=n_streams, max_batch=max_batch,
                        max_batch_bytes=max_bytes, producer_wait=False, queue_only=queue_only,
                        launch_depth=depth)
        tickets = (ctypes.c_uint64 * n)()
        lag = (ctypes.c_double * n)()
        check(cs, G.conv_loadgen_serve(srv._h, n, arr, pin, pout, kk, imgs, hs, tickets, lag))
        srv.drain()
        times = [srv.poll(t) for t in tickets]
        st = srv.stats()
        srv.destroy()
        w = times[warm:]
        mean = lambda a, b: sum(t[b] - t[a] for t in w) / len(w) / 1e3  # noqa: E731
        stages = {"queue_us": mean("submit_ns", "admit_ns"), "enqueue_us": mean("admit_ns", "launch_ns"),
                  "device_us": mean("launch_ns", "done_ns"),
                  "mean_batch": sum(t["batch_size"] for t in w) / len(w)}
        return summarize([t["submit_ns"] for t in times], [t["done_ns"] for t in times], list(lag),
                         n, warm, rate, {"launches": st["launches"],
                                         "direct_launches": st["direct_launches"],
                                         "max_batch_seen": st["max_batch"],
                                         "max_streams_busy": st["max_streams_busy"],
                                         "mean_stages": stages})

    def run_direct(n_streams, rate, n, warm, seed=5):
        arr, pin, pout, kk, imgs = requests(n, rate, seed)
        sub, done = (ctypes.c_uint64 * n)(), (ctypes.c_uint64 * n)()
        lag = (ctypes.c_double * n)()
        check(cs, G.conv_loadgen_direct(n, arr, pin, pout, kk, imgs, n_streams, sub, done, lag))
        return summarize(list(sub), list(done), list(lag), n, warm, rate, {"launches": n})

    MB = 1 << 20
    # "batched" is the server as recommended: every launch made by its
    # scheduler thread, so one thread makes all HIP calls (measured faster
    # than letting the submitting thread launch, whose launch calls then
    # contend with the scheduler's event polling in the HIP runtime)
    policies = {
        "batched": lambda rate, n, warm: run_server(16, 4, 128 * MB, rate, n, warm, queue_only=True),
        "batched_submit_launch": lambda rate, n, warm: run_server(16, 4, 128 * MB, rate, n, warm),
        "batched_8_streams": lambda rate, n, warm: run_server(16, 8, 128 * MB, rate, n, warm,
                                                              queue_only=True),
        "batched_count_cap_only": lambda rate, n, warm: run_server(16, 4, 0, rate, n, warm,
                                                                   queue_only=True),
        "batched_depth_2": lambda rate, n, warm: run_server(16, 4, 128 * MB, rate, n, warm,
                                                            queue_only=True, depth=2),
        "per_image_launch": lambda rate, n, warm: run_direct(1, rate, n, warm),
        "per_image_launch_4_streams": lambda rate, n, warm: run_direct(4, rate, n, warm),
    }
    # capacity: every request submitted at once; one untimed pass per policy
    # (a server's or a buffer set's first use runs several times slower), then
    # the median of three
    caps = {}
    for name, fn in policies.items():
        fn(0.0, 2000, 0)
        caps[name] = sorted(fn(0.0, 2000, 0)["throughput_req_per_s"] for _ in range(3))[1]
    capacity = caps["batched"]
    out = {"capacity_req_per_s": caps,
           "batched_policy": {"max_batch": 16, "streams": 4, "max_slots": NBUF,
                              "max_batch_bytes": 128 * MB, "hbm_budget_bytes": budget,
                              "launches": "scheduler thread only"},
           "sizes": [f"3x{h}x{w}" for (h, w) in sizes], "reps": args.serve_reps, "levels": {}}
    n = args.serve_requests + args.serve_warmup
    names = list(policies)
    med = lambda v: sorted(v)[len(v) // 2]  # noqa: E731
    for frac in (0.5, 0.8):
        lam = frac * capacity
        runs = {name: [] for name in names}
        # the policies take turns, in a rotated order each repetition, so that a
        # drift of the machine during the measurement falls on all of them
        for rep in range(max(1, args.serve_reps)):
            for j in range(len(names)):
                name = names[(j + rep) % len(names)]
                runs[name].append(policies[name](lam, n, args.serve_warmup))
        lvl = {"rate_req_per_s": lam}
        for name, rs in runs.items():
            r = dict(rs[len(rs) // 2])  # stage times and counters of one repetition
            r.update({"p50_us": med([x["p50_us"] for x in rs]), "p99_us": med([x["p99_us"] for x in rs]),
                      "mean_us": med([x["mean_us"] for x in rs]),
                      "p50_from_submit_us": med([x["p50_from_submit_us"] for x in rs]),
                      "p99_from_submit_us": med([x["p99_from_submit_us"] for x in rs]),
                      "per_rep_p50_p99_us": [[x["p50_us"], x["p99_us"]] for x in rs]})
            lvl[name] = r
        out["levels"][f"{frac:.1f}x_batched_capacity"] = lvl
    return out


def cpu_model() -> str:
    """The host CPU's model name (lscpu's 'Model name'), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(oracle, np, synth, host, k, args):
    """The FP64 oracle (direct 25-term sum, OpenMP over plane x row) on the
    host: the 3x4096x4096 image on every core the oracle's OpenMP team has and
    on one core, and the 64-image batch on every core and (a sample of 16 of
    its images) on one core; median of 3 runs each (the all-core image repeated
    until --cpu-min-s / 3 has passed)."""
    def med(fn, min_s=0.0, reps=3):
        times = []
        t_start = time.perf_counter()
        while len(times) < reps or (time.perf_counter() - t_start < min_s and len(times) < 200):
            t = time.perf_counter()
            fn()
            times.append(time.perf_counter() - t)
        times.sort()
        return times[len(times) // 2], len(times)

    A64 = host.astype(np.float64)
    k64 = k.astype(np.float64)
    team = oracle.max_threads()
    t_all, n_all = med(lambda: oracle.conv5(A64, k64, nthreads=0), args.cpu_min_s / 3)
    t_one, n_one = med(lambda: oracle.conv5(A64, k64, nthreads=1))
    shapes = synth.batch_shapes(3, 64)
    imgs = [(synth.image(100 + i, 3, h, w).astype(np.float64), synth.taps_random(200 + i).astype(np.float64))
            for i, (h, w) in enumerate(shapes)]
    pix = sum(h * w for h, w in shapes)
    sample = imgs[::4]
    spix = sum(a.shape[1] * a.shape[2] for a, _ in sample)

    def batch(items, nt):
        for a, kb in items:
            oracle.conv5(a, kb, nthreads=nt)

    b_all, _ = med(lambda: batch(imgs, 0))
    b_one, _ = med(lambda: batch(sample, 1))
    return {
        "value": (R * C) / t_all / 1e6,
        "unit": "MPix/s",
        "cores": team,
        "kind": "oracle",
        "sample": f"whole 3x{R}x{C} FP32 image (as FP64), FP64 direct 25-term oracle, OpenMP over "
                  f"plane x row on {team} threads, median of {n_all} runs ({t_all:.3f} s each)",
        "cpu_model": cpu_model(),
        "one_core_mpix_per_s": (R * C) / t_one / 1e6,
        "batch64_mpix_per_s": pix / b_all / 1e6,
        "batch64_one_core_mpix_per_s": spix / b_one / 1e6,
        "batch64_one_core_sample": f"16 of the 64 images (every 4th, {spix / 1e6:.1f} MPix)",
    }


def r3(x):
    """Rounds for the headline line: 4 significant digits."""
    return None if x is None else float(f"{x:.4g}")


def cfg_str(c):
    """A tile configuration in one short string."""
    return ("rows{rows_per_tile} waves{waves_per_wg} persist{persist_wgs_per_cu} "
            "xcd{xcd_slabs} pack{pack_tail}").format(**c)


def summarize(forms, extras, eq):
    """The compact per-configuration figures that go into the headline line;
    everything else goes to the detail output."""
    us = lambda v: r3(v * 1e3)  # noqa: E731  (ms -> us)
    out = {
        "c2_us": {n: us(v["ms_per_step"]) for n, v in forms.items()},
        # against the problem's 8 B per plane-pixel (read once, write once) for every form
        "c2_frac_hbm_8B": {n: r3(v["frac_of_hbm_peak"]) for n, v in forms.items()},
        # the two-pass on its own 16 B (intermediate mostly from the Infinity Cache)
        "c2_2pass_memsys_frac_16B": r3(forms.get("2pass", {}).get("own_bytes_frac_of_peak")),
        "fused_equals_2pass_bitwise": eq,
    }
    f = forms.get("fused", {})
    out["fused_frac_of_library_copy"] = r3(f.get("frac_of_copy"))
    out["fused_frac_of_torch_copy"] = r3(f.get("frac_of_torch_copy"))
    if "warm_same_buffers_avg_launch_ms" in f:
        out["fused_us_cold_warm"] = [us(f["avg_launch_ms"]), us(f["warm_same_buffers_avg_launch_ms"])]
    sm = extras.get("small")
    if sm:
        rs = sm["results"]
        out["c1_us_per_call"] = {"cols": "gpu_cold, gpu_warm, host_roundtrip",
                                 **{n: [r3(v.get("gpu_us_cold")), r3(v["gpu_us_warm"]), r3(v["host_us"])]
                                    for n, v in rs.items()}}
        out["c1_compute_us_warm"] = {n: r3(v["compute_gpu_us_warm"]) for n, v in rs.items()
                                     if "compute_gpu_us_warm" in v}
    pr = extras.get("precision")
    if pr:
        out["c4_us_per_image"] = {d: {n: us(v["ms_per_step"]) for n, v in r.items()} for d, r in pr.items()}
        out["c4_fused_frac_of_hbm_peak"] = {d: r3(r["fused"]["frac_of_hbm_peak"]) for d, r in pr.items()}
    b = extras.get("batch")
    if b:
        out["c3_batch64"] = {
            "f32": {"eager_ms": r3(b["eager_ms"]), "graph_ms": r3(b.get("graph_ms")),
                    "per_image_ms": r3(b["per_image_launches_ms"]), "tuned_ms": r3(b["tuned_eager_ms"]),
                    "frac": r3(b["eager_frac_of_hbm_peak"]), "graph_frac": r3(b.get("graph_frac_of_hbm_peak")),
                    "tuned_cfg": cfg_str(b["tuned_cfg"]), "default_cfg": cfg_str(b["tile_cfg"])},
            **{d: {"eager_ms": r3(v["eager_ms"]), "per_image_ms": r3(v["per_image_launches_ms"]),
                   "tuned_ms": r3(v["tuned_eager_ms"]), "frac": r3(v["eager_frac_of_hbm_peak"])}
               for d, v in b["16bit"].items()},
        }
    for key, name in (("serving", "c5_mixed"), ("serving_small_frames", "c5_640x480")):
        sv = extras.get(key)
        if not sv:
            continue
        pol = {"batched": "batched", "per_image_launch": "per_image_1s",
               "per_image_launch_4_streams": "per_image_4s"}
        o = {"capacity_req_per_s": {a: r3(sv["capacity_req_per_s"][p]) for p, a in pol.items()}}
        for lvl, d in sv["levels"].items():
            o[lvl.split("_")[0] + "_p50_p99_us"] = {a: [r3(d[p]["p50_us"]), r3(d[p]["p99_us"])]
                                                   for p, a in pol.items()}
        out[name] = o
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the "
              "convolution of one image is a single-GPU kernel, and sharding one image "
              "over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1711_09791_amd as cs
    from paper_1711_09791_amd import synth

    torch.cuda.set_device(0)
    host = synth.image(1, P, R, C)
    k = synth.taps_random(2)
    forms_list = [f for f in args.forms.split(",") if f]
    forms, eq = bench_image(torch, cs, host, k, args, forms=forms_list)
    progress("forms: " + ", ".join(f"{n} {v['avg_launch_ms'] * 1e3:.1f} us" for n, v in forms.items()))

    extras = {}
    want = set() if args.no_extras else {e for e in args.extras.split(",") if e}
    if "small" in want:
        extras["small"] = bench_small(torch, cs, synth, args)
        progress("small (3x256x256) done")
    if "precision" in want:
        prec = {}
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            r, _ = bench_image(torch, cs, host, k, args, dtype=dt,
                               forms=("fused", "direct25", "2pass", "2pass_t16"))
            prec[name] = r
        extras["precision"] = prec
        progress("precision done")
    if "widths" in want:
        extras["widths"] = bench_widths(torch, cs, synth, host, args)
        progress("widths done")
    if "hwc" in want:
        extras["hwc"] = bench_hwc(torch, cs, host, k, args)
        progress("hwc done")
    if "pyramid" in want:
        extras["pyramid"] = bench_pyramid(torch, cs, host, k, args)
        progress("pyramid done")
    if "batch" in want:
        extras["batch"] = bench_batch(torch, cs, synth, args)
        progress("batch done")
    if "serving" in want:
        extras["serving"] = bench_serving(torch, cs, synth, args)
        progress("serving (mixed frames) done")
        extras["serving_small_frames"] = bench_serving(torch, cs, synth, args, sizes=[(480, 640)])
        progress("serving (small frames) done")

    main_form = "fused"
    f = forms[main_form]
    cfg = cs.conv_get_tile_cfg(0, 0).as_dict()
    roofline = {
        "bound": "hbm",
        "achieved": r3(f["alg_GBps"]),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": r3(f["alg_GBps"] / HBM_PEAK_GBS),
        "traffic": traffic_for(main_form),
        "kernel": "k_image<F32, aligned, FUSED> ({rows_per_tile}-row bands, {waves_per_wg} wave(s) per "
                  "workgroup, XCD chunks of {xcd_slabs} bands)".format(**cfg),
        "alg_bytes_per_launch": f["alg_bytes_per_step"],
    }
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        cpu = cpu_baseline(oracle, np, synth, host, k, args)
        progress("cpu baseline done")
        for key in ("value", "one_core_mpix_per_s", "batch64_mpix_per_s", "batch64_one_core_mpix_per_s"):
            cpu[key] = r3(cpu[key])

    line = {
        "metric": "MPix/s (3-plane) + % HBM roofline; serving p50/p99 latency vs per-image launch",
        "value": r3(f["mpix_per_s"]),
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"one 3x{R}x{C} FP32 image, width-5 separable convolution, fused "
                        "single-pass, 2-px border 0 (uniform [0,1) pixels seed 1; positive random "
                        "taps summing to 1, seed 2)",
            "buffer_sets_rotated": max(1, args.sets),
            "tile_cfg": cfg,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "summary": summarize(forms, extras, eq),
    }
    detail = {"forms": forms, "fused_equals_2pass_bitwise": eq, **extras,
              "device": torch.cuda.get_device_name(0), "headline": dict(line)}
    detail["headline"].pop("summary")
    text = json.dumps(detail)
    if args.detail_out:
        with open(args.detail_out, "w") as fh:
            fh.write(text + "\n")
    else:
        print("bench detail: " + text, file=sys.stderr, flush=True)
    print(headline_text(line), flush=True)


HEADLINE_MAX_CHARS = 4000


def headline_text(line: dict) -> str:
    """The headline line as JSON, short enough for a log tail: summary parts are
    dropped (they remain in the detail output) until it fits."""
    out = json.dumps(line)
    for key in ("c5_640x480", "c4_us_per_image", "c1_us_per_call", "c5_mixed", "c3_batch64"):
        if len(out) <= HEADLINE_MAX_CHARS:
            break
        line["summary"].pop(key, None)
        out = json.dumps(line)
    return out


if __name__ == "__main__":
    main()
