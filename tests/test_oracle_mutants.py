"""Plant mistakes in copies of the oracle (on the CPU) and check the pins catch
each one.  This shows the pins are discriminating: a dropped term, a flipped
or wrong index, a wrong sign or border, or a row pass that skips the outer
rows (the literal reading of the OpenMP listing of Section 5.3) all fail at
least one pin.  Nothing here touches a GPU.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests import oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "conv5_oracle.c")

# (name, function the mistake lands in, original text, replacement)
MUTANTS = [
    ("flipped_kernel", "direct",
     "acc += Ap[(y + a) * cols + (x + b)] * Kab;",
     "acc += Ap[(y - a) * cols + (x - b)] * Kab;"),
    ("flipped_columns", "direct",
     "acc += Ap[(y + a) * cols + (x + b)] * Kab;",
     "acc += Ap[(y + a) * cols + (x - b)] * Kab;"),
    ("dropped_tap", "direct",
     "for (int b = -R5; b <= R5; ++b) {",
     "for (int b = -R5; b < R5; ++b) {"),
    ("wrong_K_index", "direct",
     "const double Kab = k[a + R5] * k[b + R5];",
     "const double Kab = k[a + R5] * k[a + R5];"),
    ("wrong_sign", "direct",
     "acc += Ap[(y + a) * cols + (x + b)] * Kab;",
     "acc -= Ap[(y + a) * cols + (x + b)] * Kab;"),
    ("border_off_by_one", "direct",
     "for (int64_t x = R5; x < cols - R5; ++x) {\n                double acc",
     "for (int64_t x = R5; x < cols - R5 - 1; ++x) {\n                double acc"),
    ("plane_offset_lost", "direct",
     "const double *Ap = A + p * plane_elems;\n            double *Bp = B + p * plane_elems;\n            for (int64_t x",
     "const double *Ap = A;\n            double *Bp = B + p * plane_elems;\n            for (int64_t x"),
    ("row_pass_interior_only", "twopass",
     "for (int64_t y = 0; y < rows; ++y)            /* horizontal pass */",
     "for (int64_t y = R5; y < rows - R5; ++y)      /* horizontal pass */"),
    ("vertical_tap_transposed", "twopass",
     "s += aux[(y + a) * cols + x] * k[a + R5];",
     "s += aux[(y + a) * cols + x] * k[R5 - a];"),
]


# Mistakes in the width-n, full-kernel function.
N_MUTANTS = [
    ("n_transposed_K",
     "acc += src[(y + a - r) * cols + (x + b - r)] * K[a * n + b];",
     "acc += src[(y + a - r) * cols + (x + b - r)] * K[b * n + a];"),
    ("n_flipped_kernel",
     "acc += src[(y + a - r) * cols + (x + b - r)] * K[a * n + b];",
     "acc += src[(y - a + r) * cols + (x - b + r)] * K[a * n + b];"),
    ("n_dropped_column",
     "for (int b = 0; b < n; ++b)",
     "for (int b = 0; b < n - 1; ++b)"),
    ("n_border_off_by_one",
     "for (int64_t x = r; x < cols - r; ++x) {",
     "for (int64_t x = r; x < cols - r - 1; ++x) {"),
    ("n_plane_offset_lost",
     "const double *src = A + p * plane_elems;",
     "const double *src = A;"),
    ("n_radius_rounded_up",
     "const int r = n / 2;",
     "const int r = (n + 1) / 2;"),
]


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} must match exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    str(path), "-o", str(so), "-lm"], check=True)
    return ctypes.CDLL(str(so))


def _wrap(lib, which):
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64

    def conv(A, k):
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        k = np.ascontiguousarray(np.asarray(k, dtype=np.float64))
        B = np.empty_like(A)
        P, R, C = A.shape
        p = lambda a: a.ctypes.data_as(dp)  # noqa: E731
        if which == "direct":
            f = lib.oracle_conv5_direct
            f.argtypes = [dp, dp, dp, i64, i64, i64, ctypes.c_int]
            f(p(A), p(B), p(k), P, R, C, 1)
        else:
            aux = np.empty((max(R * C, 1),))
            f = lib.oracle_conv5_twopass
            f.argtypes = [dp, dp, dp, dp, i64, i64, i64]
            f(p(A), p(B), p(aux), p(k), P, R, C)
        return B

    return conv


@pytest.mark.parametrize("name,which,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_mutant(tmp_path, name, which, old, new):
    lib = _build_mutant(tmp_path, name, old, new)
    bad = pins.failing_pins(_wrap(lib, which))
    assert bad, f"mutant {name} passed every pin"


def test_unmutated_copy_passes(tmp_path):
    lib = _build_mutant(tmp_path, "identity", "#define R5 2", "#define R5 2")
    assert pins.failing_pins(_wrap(lib, "direct")) == []
    assert pins.failing_pins(_wrap(lib, "twopass")) == []


ROUND_MUTANTS = [
    ("ties_away", "if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) != 0.0))",
     "if (rem >= 0.5)"),
    ("truncate", "if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) != 0.0))",
     "if (0)"),
]


@pytest.mark.parametrize("name,old,new", ROUND_MUTANTS, ids=[m[0] for m in ROUND_MUTANTS])
def test_rounding_pins_reject_mutant(tmp_path, name, old, new):
    lib = _build_mutant(tmp_path, name, old, new)
    u16p = ctypes.POINTER(ctypes.c_uint16)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_round_f16.argtypes = [dp, u16p, ctypes.c_int64]
    h = np.arange(0, 0x7bff, 7, dtype=np.uint16)
    a = h.view(np.float16).astype(np.float64)
    b = (h + 1).astype(np.uint16).view(np.float16).astype(np.float64)
    v = np.ascontiguousarray(np.concatenate([(a + b) / 2, a + (b - a) * 0.7]))
    out = np.empty(v.shape, dtype=np.uint16)
    lib.oracle_round_f16(v.ctypes.data_as(dp), out.ctypes.data_as(u16p), v.size)
    assert not np.array_equal(out, v.astype(np.float16).view(np.uint16))


def _wrap_n(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    f = lib.oracle_conv_direct_n
    f.argtypes = [dp, dp, dp, ctypes.c_int, i64, i64, i64, ctypes.c_int]

    def convK(A, K):
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        K = np.ascontiguousarray(np.asarray(K, dtype=np.float64))
        B = np.empty_like(A)
        P, R, C = A.shape
        p = lambda a: a.ctypes.data_as(dp)  # noqa: E731
        f(p(A), p(B), p(K), int(K.shape[0]), P, R, C, 1)
        return B

    return convK


@pytest.mark.parametrize("name,old,new", N_MUTANTS, ids=[m[0] for m in N_MUTANTS])
def test_n_pins_reject_mutant(tmp_path, name, old, new):
    lib = _build_mutant(tmp_path, name, old, new)
    assert pins.failing_n_pins(_wrap_n(lib)), f"mutant {name} passed every pin"


def test_n_unmutated_copy_passes(tmp_path):
    lib = _build_mutant(tmp_path, "identity_n", "#define R5 2", "#define R5 2")
    assert pins.failing_n_pins(_wrap_n(lib)) == []


# Mistakes in the two-pass form with a 16-bit intermediate (C code).
Q_MUTANTS = [
    ("q_not_rounded",
     "for (int64_t e = 0; e < n_plane; ++e)",
     "for (int64_t e = 0; e < 0; ++e)"),
    ("q_formats_swapped",
     "aux[e] = tfmt == 1 ? half_bits_to_double",
     "aux[e] = tfmt == 2 ? half_bits_to_double"),
    ("q_interior_rows_rounded_only",
     "for (int64_t e = 0; e < n_plane; ++e)",
     "for (int64_t e = R5 * cols; e < n_plane - R5 * cols; ++e)"),
    ("q_row_pass_interior_only",
     "for (int64_t i = 0; i < rows; ++i)\n            for (int64_t j = R5; j < cols - R5; ++j) {\n                double h",
     "for (int64_t i = R5; i < rows - R5; ++i)\n            for (int64_t j = R5; j < cols - R5; ++j) {\n                double h"),
    ("q_vertical_tap_flipped",
     "v += aux[(i + d) * cols + j] * k[d + R5];",
     "v += aux[(i + d) * cols + j] * k[R5 - d];"),
]


def _wrap_q(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    f = lib.oracle_conv5_twopass_q
    f.argtypes = [dp, dp, dp, dp, i64, i64, i64, ctypes.c_int]

    def conv_t(A, k, fmt):
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        k = np.ascontiguousarray(np.asarray(k, dtype=np.float64))
        B = np.empty_like(A)
        P, R, C = A.shape
        aux = np.empty((max(R * C, 1),))
        p = lambda a: a.ctypes.data_as(dp)  # noqa: E731
        f(p(A), p(B), p(aux), p(k), P, R, C, {"f16": 1, "bf16": 2}[fmt])
        return B

    return conv_t


@pytest.mark.parametrize("name,old,new", Q_MUTANTS, ids=[m[0] for m in Q_MUTANTS])
def test_t16_pins_reject_c_mutant(tmp_path, name, old, new):
    lib = _build_mutant(tmp_path, name, old, new)
    assert pins.failing_t16_pins(_wrap_q(lib)), f"mutant {name} passed every pin"


def test_t16_unmutated_copy_passes(tmp_path):
    lib = _build_mutant(tmp_path, "identity_q", "#define R5 2", "#define R5 2")
    assert pins.failing_t16_pins(_wrap_q(lib)) == []
