#!/usr/bin/env python3
"""Throughput of the width-5 separable convolution on one MI355X.

Workload: one 3-plane 4096 x 4096 FP32 image (uniform [0,1) pixels, seed 1),
positive random taps normalised to sum 1 (seed 2); 2-pixel border = 0.
A step is one fused single-pass convolution of the image (input read, row
filter, on-chip intermediate, column filter, border, output store).  The
two-pass form (HBM intermediate) and the direct 25-tap form are timed the same
way and reported under "forms"; a device copy of the same bytes is the
achievable ceiling.  Inputs are resident in HBM; the timed launches rotate over
several input/output buffer sets so the working set exceeds the 256 MB
Infinity Cache.

Prints ONE JSON line.  Run with no flags for the default configuration.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_DIR = os.path.join(ROOT, "paper_1711_09791_amd", "csrc")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sets", type=int, default=3, help="rotating buffer sets")
    ap.add_argument("--forms", default="fused,2pass,direct25,copy")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-min-s", type=float, default=10.0,
                    help="repeat the oracle until this much CPU time is spent")
    return ap.parse_args()


def kernel_src_sha() -> str:
    """sha256 over the device-code sources (conv_kernels*.{h,hip}, conv_internal.h)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_DIR)):
        if name.startswith("conv_kernels") or name == "conv_internal.h":
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the "
              "convolution of one image is a single-GPU kernel; multi-GPU sharding is "
              "described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1711_09791_amd as cs
    from paper_1711_09791_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    host = synth.image(1, P, R, C)
    k = synth.taps_random(2)
    base = torch.from_numpy(host).to(dev)
    S = max(1, args.sets)
    ins = [base] + [base.clone() for _ in range(S - 1)]
    outs = [torch.empty_like(base) for _ in range(S)]
    tmp = torch.empty(P * R * C, device=dev)
    stream = torch.cuda.current_stream()

    # Prepared C-ABI arguments: the timed loop makes one foreign call per step.
    L = cs.lib()
    img = cs.image_of(base)
    kk = (ctypes.c_float * 5)(*[float(v) for v in k])
    hs = ctypes.c_void_p(stream.cuda_stream)
    pin = [ctypes.c_void_p(t.data_ptr()) for t in ins]
    pout = [ctypes.c_void_p(t.data_ptr()) for t in outs]
    ptmp = ctypes.c_void_p(tmp.data_ptr())
    pimg = ctypes.byref(img)

    def call(st):
        if st != 0:
            raise cs.ConvError(st, cs.conv_last_error())

    steps_fn = {
        "fused": lambda i: call(L.conv_sep5_1pass(pin[i % S], pout[i % S], kk, pimg, 0, hs)),
        "direct25": lambda i: call(L.conv_sep5_1pass(pin[i % S], pout[i % S], kk, pimg, 1, hs)),
        "2pass": lambda i: call(L.conv_sep5_2pass(pin[i % S], pout[i % S], ptmp, kk, pimg, hs)),
        "copy": lambda i: outs[i % S].copy_(ins[i % S]),
    }
    alg_bytes = {  # algorithmic HBM bytes per step
        "fused": 8 * P * R * C, "direct25": 8 * P * R * C, "2pass": 16 * P * R * C,
        "copy": 8 * P * R * C,
    }

    def timed(fn, steps, warmup):
        for i in range(warmup):
            fn(i)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for i in range(steps):
            ev[i][0].record()
            fn(i)
            ev[i][1].record()
        t1.record()
        torch.cuda.synchronize()
        total = t0.elapsed_time(t1)
        per = sorted(a.elapsed_time(b) for a, b in ev)
        return total, per

    forms = {}
    for name in [f for f in args.forms.split(",") if f]:
        total, per = timed(steps_fn[name], args.steps, args.warmup)
        avg = sum(per) / len(per)
        forms[name] = {
            "ms_per_step": total / args.steps,
            "avg_launch_ms": avg,
            "median_launch_ms": per[len(per) // 2],
            "mpix_per_s": (R * C) / (total / args.steps * 1e-3) / 1e6,
            "alg_GBps": alg_bytes[name] / (avg * 1e-3) / 1e9,
            "frac_of_hbm_peak": alg_bytes[name] / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
    # warm number for the fused form: the same buffer set every step
    if "fused" in forms:
        fn = lambda i: call(L.conv_sep5_1pass(pin[0], pout[0], kk, pimg, 0, hs))  # noqa: E731
        total, per = timed(fn, args.steps, args.warmup)
        forms["fused"]["warm_same_buffers_avg_launch_ms"] = sum(per) / len(per)
    if "copy" in forms and "fused" in forms:
        forms["fused"]["frac_of_copy"] = forms["copy"]["avg_launch_ms"] / forms["fused"]["avg_launch_ms"]

    # consistency of the timed outputs: fused and two-pass are bitwise equal
    check = None
    if "fused" in forms and "2pass" in forms:
        o1, o2 = torch.empty_like(base), torch.empty_like(base)
        cs.conv_sep5_1pass(base, o1, k)
        cs.conv_sep5_2pass(base, o2, k, d_tmp=tmp)
        torch.cuda.synchronize()
        check = bool(torch.equal(o1, o2))

    main_form = "fused"
    f = forms[main_form]
    traffic = traffic_for(main_form)
    roofline = {
        "bound": "hbm",
        "achieved": f["alg_GBps"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": f["alg_GBps"] / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": "fused single-pass FP32 (k_image<F32,aligned,FUSED>)",
        "alg_bytes_per_launch": alg_bytes[main_form],
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        A64 = host.astype(np.float64)
        k64 = k.astype(np.float64)
        times = []
        t_start = time.perf_counter()
        while (len(times) < 3 or time.perf_counter() - t_start < args.cpu_min_s) \
                and len(times) < 200:
            t = time.perf_counter()
            oracle.conv5(A64, k64, nthreads=0)
            times.append(time.perf_counter() - t)
            if time.perf_counter() - t_start > 3 * args.cpu_min_s:
                break
        times.sort()
        med = times[len(times) // 2]
        cpu = {
            "value": (R * C) / med / 1e6,
            "unit": "MPix/s",
            "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"whole 3x{R}x{C} image, FP64 direct 25-term oracle (OpenMP over "
                      f"plane x row), median of {len(times)} run(s), {med:.3f} s each",
        }

    ms = forms[main_form]["ms_per_step"]
    line = {
        "metric": "MPix/s (3-plane) + % HBM roofline; serving p50/p99 latency vs per-image launch",
        "value": forms[main_form]["mpix_per_s"],
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"one 3x{R}x{C} FP32 image, width-5 separable convolution, fused "
                        "single-pass, 2-px border 0",
            "planes": P, "rows": R, "cols": C,
            "taps": "positive random, normalised to sum 1 (seed 2)",
            "pixels": "uniform [0,1) (seed 1)",
            "buffer_sets_rotated": S,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "fused_equals_2pass_bitwise": check,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
