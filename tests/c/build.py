"""Compiles abi_check.c (a plain-C user of the C ABI, linked with the C
oracle as test infrastructure) into tests/c/abi_check.  Called by the
repository's build step after libconvsep5.so is built."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(HERE, "abi_check")


def build() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = [
        "gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
        f"-I{rocm}/include", f"-I{ROOT}/include",
        os.path.join(HERE, "abi_check.c"), os.path.join(ROOT, "oracle", "conv5_oracle.c"),
        f"-L{ROOT}/paper_1711_09791_amd", "-lconvsep5", f"-L{rocm}/lib", "-lamdhip64", "-lm",
        "-Wl,-rpath,$ORIGIN/../../paper_1711_09791_amd", f"-Wl,-rpath,{rocm}/lib",
        "-o", BIN,
    ]
    subprocess.run(cmd, check=True)
    return BIN


if __name__ == "__main__":
    print(build())
