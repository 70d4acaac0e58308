"""The C ABI from plain C (tests/c/abi_check.c): HIP device memory, every
width-5 form and a batch against the FP64 oracle, no Python in the path."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_check")


def test_c_program_against_oracle():
    if not os.path.exists(BIN):
        pytest.fail("tests/c/abi_check is not built (run the build step)")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi_check OK" in r.stdout
