"""Build libconvsep5.so in-tree with hipcc for gfx950.

    python -m paper_1711_09791_amd.build          # compile (always)
    python -m paper_1711_09791_amd.build --incremental   # only what changed

Each translation unit is compiled to an object in parallel, then linked into
``paper_1711_09791_amd/libconvsep5.so``.  Device code is built with FP
contraction off (every multiply-add in the kernels is an explicit fma) and
with the packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libconvsep5.so")
LOADGEN_LIB = os.path.join(PKG, "libconvsep5_loadgen.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["conv_kernels_f32.hip", "conv_kernels_f16.hip", "conv_kernels_bf16.hip",
           "conv_kernels_n_f32.hip", "conv_kernels_n_f16.hip", "conv_kernels_n_bf16.hip",
           "conv_kernels_pyr.hip", "conv_kernels_hwc.hip",
           "conv_api.cpp", "conv_api_n.cpp", "conv_api_pyr.cpp", "conv_tune.cpp", "conv_serve.cpp"]
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > _headers_mtime():
            return obj
    cmd = [_hipcc(), *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source and link libconvsep5.so.  By default everything
    is recompiled; incremental=True reuses objects newer than their source and
    every header."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    # the serving load generator: a separate library on top of the public ABI
    obj = _compile("conv_loadgen.cpp", incremental)
    tmp = LOADGEN_LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", obj, "-o", tmp,
           f"-L{PKG}", "-lconvsep5", "-Wl,-rpath,$ORIGIN", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed (loadgen):\n{r.stderr}")
    os.replace(tmp, LOADGEN_LIB)
    if verbose:
        print("built", LIB, "and", LOADGEN_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
