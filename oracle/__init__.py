"""FP64 CPU oracle for the width-5 separable convolution (arXiv 1711.09791).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The
product library neither imports nor links it, and it imports nothing from
the product package: the two paths share no code.

The arithmetic lives in ``conv5_oracle.c`` (plain binary64 loops); this module
only compiles it with gcc (on first use, if it is not built yet) and marshals
numpy arrays through ctypes.

Functions (all follow Eq. 1 of Section 1 with K = k k^T, the border rule of
Section 5's opening paragraph, and planes processed independently as in the
per-plane driver of Section 5.3):

``conv5(A, k)``            single-pass (25-term) form in FP64.
``conv5_twopass(A, k)``    separable two-pass form in FP64.
``conv5_twopass_t(A, k, t)``  the two-pass form with its auxiliary array (the
                           intermediate) rounded once to t = "f16" or "bf16"
                           (RNE) between the passes; "f32" is conv5_twopass.
``conv_direct_n(A, K)``    Eq. 1 at odd width n with a full n x n kernel K.
``conv_sep_n(A, k)``       the same with K = k k^T (products in FP64, exact).
``pyr_down(A, k)``         one pyramid level: conv5, then every second row and
                           column (a reading: the paper names image scaling in
                           Section 1 but does not define it).
``decode(bits, dtype)``    exact FP32 / FP16 / BF16 storage -> float64.
``round_to(x, dtype)``     float64 -> FP16 / BF16 bits, one RNE rounding.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "conv5_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile conv5_oracle.c into _liboracle.so with gcc (OpenMP on)."""
    if force or not os.path.exists(_LIB) or (
        os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = [
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
            "-fno-fast-math", "-ffp-contract=off", "-D_GNU_SOURCE",
            _SRC, "-o", tmp, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    u16p = ctypes.POINTER(ctypes.c_uint16)
    fp = ctypes.POINTER(ctypes.c_float)
    i64 = ctypes.c_int64
    lib.oracle_conv5_direct.argtypes = [dp, dp, dp, i64, i64, i64, ctypes.c_int]
    lib.oracle_conv5_direct.restype = None
    lib.oracle_conv5_twopass.argtypes = [dp, dp, dp, dp, i64, i64, i64]
    lib.oracle_conv5_twopass.restype = None
    lib.oracle_conv5_twopass_q.argtypes = [dp, dp, dp, dp, i64, i64, i64, ctypes.c_int]
    lib.oracle_conv5_twopass_q.restype = None
    lib.oracle_conv_direct_n.argtypes = [dp, dp, dp, ctypes.c_int, i64, i64, i64, ctypes.c_int]
    lib.oracle_conv_direct_n.restype = None
    lib.oracle_decode_f32.argtypes = [fp, dp, i64]
    lib.oracle_decode_f16.argtypes = [u16p, dp, i64]
    lib.oracle_decode_bf16.argtypes = [u16p, dp, i64]
    lib.oracle_round_f16.argtypes = [dp, u16p, i64]
    lib.oracle_round_bf16.argtypes = [dp, u16p, i64]
    for f in ("oracle_decode_f32", "oracle_decode_f16", "oracle_decode_bf16",
              "oracle_round_f16", "oracle_round_bf16"):
        getattr(lib, f).restype = None
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_last_team.argtypes = []
    lib.oracle_last_team.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_planes(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    if A.ndim == 2:
        A = A[None]
    if A.ndim != 3:
        raise ValueError("image must be [planes, rows, cols] or [rows, cols]")
    return np.ascontiguousarray(A)


def _taps(k) -> np.ndarray:
    k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1))
    if k.shape != (5,):
        raise ValueError("k must hold 5 taps")
    return k


def conv5(A, k, nthreads: int = 1) -> np.ndarray:
    """Eq. 1 with K[i][j] = k_i k_j, 25 FP64 terms per interior pixel.

    A: [planes, rows, cols] (or [rows, cols]) real array, decoded to float64.
    k: 5 taps; k[0] weights the neighbour at offset -2 (correlation form).
    Returns float64 of A's shape with the 2-pixel border equal to 0.
    """
    squeeze = np.asarray(A).ndim == 2
    A = _as_planes(A)
    k = _taps(k)
    B = np.empty_like(A)
    P, R, C = A.shape
    _load().oracle_conv5_direct(_ptr(A, ctypes.c_double), _ptr(B, ctypes.c_double),
                                _ptr(k, ctypes.c_double), P, R, C, int(nthreads))
    return B[0] if squeeze else B


def conv5_twopass(A, k) -> np.ndarray:
    """Separable two-pass form (row pass on every row, then column pass), FP64."""
    squeeze = np.asarray(A).ndim == 2
    A = _as_planes(A)
    k = _taps(k)
    B = np.empty_like(A)
    P, R, C = A.shape
    aux = np.empty((max(R * C, 1),), dtype=np.float64)
    _load().oracle_conv5_twopass(_ptr(A, ctypes.c_double), _ptr(B, ctypes.c_double),
                                 _ptr(aux, ctypes.c_double), _ptr(k, ctypes.c_double),
                                 P, R, C)
    return B[0] if squeeze else B


def conv5_twopass_t(A, k, tdtype: str) -> np.ndarray:
    """Two-pass form with a 16-bit intermediate: exact row pass on every row,
    each intermediate value rounded once (RNE) to tdtype ("f16" or "bf16"),
    exact column pass over the rounded values; border 0.  "f32" gives
    conv5_twopass (the FP64 intermediate, unrounded)."""
    if tdtype == "f32":
        return conv5_twopass(A, k)
    fmt = {"f16": 1, "bf16": 2}[tdtype]
    squeeze = np.asarray(A).ndim == 2
    A = _as_planes(A)
    k = _taps(k)
    B = np.empty_like(A)
    P, R, C = A.shape
    aux = np.empty((max(R * C, 1),), dtype=np.float64)
    _load().oracle_conv5_twopass_q(_ptr(A, ctypes.c_double), _ptr(B, ctypes.c_double),
                                   _ptr(aux, ctypes.c_double), _ptr(k, ctypes.c_double),
                                   P, R, C, fmt)
    return B[0] if squeeze else B


def conv_direct_n(A, K, nthreads: int = 1) -> np.ndarray:
    """Eq. 1 at odd width n with a full (not necessarily separable) kernel.

    K: [n, n], n odd in 1..; K[a, b] weights A[y + a - n//2, x + b - n//2].
    Returns float64 of A's shape with the (n//2)-pixel border equal to 0.
    """
    squeeze = np.asarray(A).ndim == 2
    A = _as_planes(A)
    K = np.ascontiguousarray(np.asarray(K, dtype=np.float64))
    if K.ndim != 2 or K.shape[0] != K.shape[1] or K.shape[0] % 2 == 0:
        raise ValueError("K must be a square matrix of odd width")
    B = np.empty_like(A)
    P, R, C = A.shape
    _load().oracle_conv_direct_n(_ptr(A, ctypes.c_double), _ptr(B, ctypes.c_double),
                                 _ptr(K, ctypes.c_double), int(K.shape[0]), P, R, C,
                                 int(nthreads))
    return B[0] if squeeze else B


def conv_sep_n(A, k, nthreads: int = 1) -> np.ndarray:
    """Eq. 1 at odd width n with the separable kernel K = k k^T.

    k holds n taps (FP32 values); their products are exact in FP64.
    """
    k = np.asarray(k, dtype=np.float64).reshape(-1)
    return conv_direct_n(A, np.outer(k, k), nthreads)


def pyr_down(A, k, nthreads: int = 1) -> np.ndarray:
    """Blur then 2x decimation: out[p, yo, xo] = conv5(A, k)[p, 2 yo, 2 xo],
    shape [planes, ceil(rows/2), ceil(cols/2)] (the zero frame of conv5 is
    sampled like every other pixel)."""
    B = conv5(A, k, nthreads)
    return np.ascontiguousarray(B[..., ::2, ::2])


def decode(bits: np.ndarray, dtype: str) -> np.ndarray:
    """Exact storage -> float64.  dtype in {"f32", "f16", "bf16"}.

    For "f32" pass float32 values; for "f16"/"bf16" pass the raw uint16 bits.
    """
    lib = _load()
    if dtype == "f32":
        src = np.ascontiguousarray(bits, dtype=np.float32)
        out = np.empty(src.shape, dtype=np.float64)
        lib.oracle_decode_f32(_ptr(src, ctypes.c_float), _ptr(out, ctypes.c_double), src.size)
        return out
    src = np.ascontiguousarray(bits).view(np.uint16)
    out = np.empty(src.shape, dtype=np.float64)
    if dtype == "f16":
        lib.oracle_decode_f16(_ptr(src, ctypes.c_uint16), _ptr(out, ctypes.c_double), src.size)
    elif dtype == "bf16":
        lib.oracle_decode_bf16(_ptr(src, ctypes.c_uint16), _ptr(out, ctypes.c_double), src.size)
    else:
        raise ValueError(dtype)
    return out


def round_to(x: np.ndarray, dtype: str) -> np.ndarray:
    """float64 -> 16-bit storage bits (uint16), one round-to-nearest-even."""
    src = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(src.shape, dtype=np.uint16)
    lib = _load()
    if dtype == "f16":
        lib.oracle_round_f16(_ptr(src, ctypes.c_double), _ptr(out, ctypes.c_uint16), src.size)
    elif dtype == "bf16":
        lib.oracle_round_bf16(_ptr(src, ctypes.c_double), _ptr(out, ctypes.c_uint16), src.size)
    else:
        raise ValueError(dtype)
    return out


def max_threads() -> int:
    """Threads an OpenMP region of the oracle uses by default on this host."""
    return int(_load().oracle_max_threads())


def last_team() -> int:
    """Threads the oracle's last parallel region asked for (its nthreads, or
    the OpenMP default for nthreads <= 0)."""
    return int(_load().oracle_last_team())
