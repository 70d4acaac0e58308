"""Pins for the FP64 oracle: checks that tie it to something other than itself.

Each pin takes a convolution callable ``conv(A, k) -> B`` (A is [P, R, C]
float64, k holds 5 taps) so the same pins can be run against deliberately
broken copies of the oracle (see test_oracle_mutants.py) and must reject them.

Sources of truth used here, none of which is the oracle:
* library routines: scipy.signal.correlate2d and torch conv2d (CPU, float64),
  which compute Eq. 1 as a correlation on the 'valid' region;
* brute force: Eq. 1 written with an explicit K[i][j] = k_i k_j matrix in
  pure Python on tiny images;
* closed forms: delta impulse, constant image, linear ramp, exact rationals;
* for the two-pass form with a 16-bit intermediate: an independent rounding
  (Python's round-half-even on the scaled value) in a brute-force loop, exact
  dyadic cases and the closed-form error bound of one rounding per value.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _interior_expected(A: np.ndarray, K: np.ndarray, valid) -> np.ndarray:
    P, R, C = A.shape
    B = np.zeros_like(A)
    if R >= 5 and C >= 5:
        for p in range(P):
            B[p, 2:R - 2, 2:C - 2] = valid(A[p], K)
    return B


def pin_scipy(conv) -> bool:
    """Eq. 1 as scipy's 2-D correlation on the 'valid' region, border 0."""
    from scipy.signal import correlate2d

    rng = np.random.default_rng(11)
    for (P, R, C) in ((3, 17, 23), (2, 40, 9), (1, 5, 5), (3, 64, 67)):
        A = rng.random((P, R, C)) * 2 - 1
        k = rng.random(5) * 2 - 1
        K = np.outer(k, k)
        ref = _interior_expected(A, K, lambda a, K: correlate2d(a, K, mode="valid"))
        got = conv(A, k)
        if got.shape != ref.shape or not np.allclose(got, ref, rtol=0, atol=1e-13):
            return False
    return True


def pin_torch(conv) -> bool:
    """Eq. 1 as torch's conv2d (a cross-correlation) in float64 on the CPU."""
    import torch

    rng = np.random.default_rng(12)
    A = rng.random((3, 33, 29)) * 2 - 1
    k = rng.random(5) * 2 - 1
    K = torch.from_numpy(np.outer(k, k))[None, None]
    t = torch.from_numpy(A)[:, None]
    valid = torch.nn.functional.conv2d(t, K)[:, 0].numpy()
    ref = np.zeros_like(A)
    ref[:, 2:-2, 2:-2] = valid
    got = conv(A, k)
    return bool(np.allclose(got, ref, rtol=0, atol=1e-13))


def _brute(a2d, k):
    R, C = len(a2d), len(a2d[0])
    K = [[k[i] * k[j] for j in range(5)] for i in range(5)]
    out = [[0.0] * C for _ in range(R)]
    for y in range(2, R - 2):
        for x in range(2, C - 2):
            s = 0.0
            for i in range(5):
                for j in range(5):
                    s += a2d[y + i - 2][x + j - 2] * K[i][j]
            out[y][x] = s
    return out


def pin_bruteforce_tiny(conv) -> bool:
    """Every H, W in 1..12 (H or W < 5 gives an all-zero result)."""
    rng = np.random.default_rng(13)
    k = rng.random(5) * 2 - 1
    for R in range(1, 13):
        for C in range(1, 13):
            A = rng.random((1, R, C)) * 2 - 1
            ref = np.array(_brute(A[0].tolist(), k.tolist()))
            got = conv(A, k)
            if got.shape != (1, R, C) or not np.allclose(got[0], ref, rtol=0, atol=1e-14):
                return False
    return True


def pin_delta(conv) -> bool:
    """A unit impulse at (y0, x0) gives B[y0+d][x0+e] = k[2-d] k[2-e]."""
    k = np.array([0.1, 0.2, 0.3, 0.4, 0.5])
    R, C, y0, x0 = 13, 15, 6, 7
    A = np.zeros((1, R, C))
    A[0, y0, x0] = 1.0
    ref = np.zeros((R, C))
    for d in range(-2, 3):
        for e in range(-2, 3):
            ref[y0 + d, x0 + e] = k[2 - d] * k[2 - e]
    got = conv(A, k)[0]
    return bool(np.array_equal(got, ref))


def pin_constant(conv) -> bool:
    """A constant image c gives c (sum k)^2 on the interior and 0 outside."""
    k = np.array([0.5, -0.25, 1.0, 0.125, 0.75])
    c = 3.0
    A = np.full((2, 9, 11), c)
    got = conv(A, k)
    ref = np.zeros_like(A)
    ref[:, 2:-2, 2:-2] = c * k.sum() ** 2
    return bool(np.allclose(got, ref, rtol=1e-15, atol=0))


def pin_ramp(conv) -> bool:
    """A = a + b y + c x with asymmetric taps (closed form, pins orientation).

    B = S^2 (a + b y + c x) + S m (b + c) with S = sum k and
    m = sum_j j k[j + 2] (first moment); a flipped (convolution-form) kernel
    would flip the sign of m.
    """
    k = np.array([0.05, 0.1, 0.15, 0.3, 0.4])
    a, b, c = 0.5, 2.0, -3.0
    R, C = 12, 14
    yy, xx = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    A = (a + b * yy + c * xx)[None].astype(np.float64)
    S = k.sum()
    m = float(np.dot(np.arange(-2, 3), k))
    ref = np.zeros_like(A)
    ref[0, 2:-2, 2:-2] = (S * S * (a + b * yy + c * xx) + S * m * (b + c))[2:-2, 2:-2]
    got = conv(A, k)
    return bool(np.allclose(got, ref, rtol=1e-13, atol=1e-13))


def pin_exact_rational(conv) -> bool:
    """m/256 pixels, binomial taps: every term is exact; compare with Fractions."""
    rng = np.random.default_rng(14)
    M = rng.integers(0, 256, size=(2, 9, 10))
    A = M / 256.0
    kf = [Fraction(v, 16) for v in (1, 4, 6, 4, 1)]
    k = np.array([float(v) for v in kf])
    got = conv(A, k)
    for p in range(2):
        for y in range(9):
            for x in range(10):
                if 2 <= y < 7 and 2 <= x < 8:
                    s = sum(Fraction(int(M[p, y + i - 2, x + j - 2]), 256) * kf[i] * kf[j]
                            for i in range(5) for j in range(5))
                else:
                    s = Fraction(0)
                if Fraction(float(got[p, y, x])) != s:
                    return False
    return True


def pin_planes_independent(conv) -> bool:
    """Each plane is convolved on its own (plane permutation commutes)."""
    rng = np.random.default_rng(15)
    A = rng.random((3, 10, 12))
    k = rng.random(5)
    B = conv(A, k)
    Bp = conv(A[[2, 0, 1]], k)
    single = [conv(A[p:p + 1], k)[0] for p in range(3)]
    return bool(np.array_equal(Bp, B[[2, 0, 1]])
                and all(np.array_equal(single[p], B[p]) for p in range(3)))


def pin_transpose(conv) -> bool:
    """K = k k^T is symmetric, so conv(A^T) = conv(A)^T."""
    rng = np.random.default_rng(16)
    A = rng.random((1, 11, 16))
    k = rng.random(5) * 2 - 1
    B = conv(A, k)[0]
    Bt = conv(np.ascontiguousarray(A[0].T)[None], k)[0]
    return bool(np.allclose(Bt, B.T, rtol=0, atol=1e-14))


def pin_linear(conv) -> bool:
    """conv(alpha A1 + beta A2) = alpha conv(A1) + beta conv(A2)."""
    rng = np.random.default_rng(17)
    A1, A2 = rng.random((2, 1, 12, 13))
    k = rng.random(5)
    lhs = conv(2.0 * A1 - 0.5 * A2, k)
    rhs = 2.0 * conv(A1, k) - 0.5 * conv(A2, k)
    return bool(np.allclose(lhs, rhs, rtol=0, atol=1e-13))


CONV_PINS = {
    "scipy": pin_scipy,
    "torch": pin_torch,
    "bruteforce_tiny": pin_bruteforce_tiny,
    "delta": pin_delta,
    "constant": pin_constant,
    "ramp": pin_ramp,
    "exact_rational": pin_exact_rational,
    "planes_independent": pin_planes_independent,
    "transpose": pin_transpose,
    "linear": pin_linear,
}


def failing_pins(conv) -> list[str]:
    bad = []
    for name, pin in CONV_PINS.items():
        try:
            ok = pin(conv)
        except Exception:
            ok = False
        if not ok:
            bad.append(name)
    return bad


# ---- pins for the width-n, full-kernel form ------------------------------
# Each takes ``convK(A, K) -> B`` with K a full [n, n] matrix (n odd).  Kernels
# are deliberately not symmetric, so a transposed or flipped K fails.

def _interior_n(A: np.ndarray, K: np.ndarray, valid) -> np.ndarray:
    P, R, C = A.shape
    n = K.shape[0]
    r = n // 2
    B = np.zeros_like(A)
    if R >= n and C >= n:
        for p in range(P):
            B[p, r:R - r, r:C - r] = valid(A[p], K)
    return B


def pin_n_scipy(convK) -> bool:
    """Eq. 1 at widths 1..9 as scipy's 2-D correlation, 'valid' region."""
    from scipy.signal import correlate2d

    rng = np.random.default_rng(31)
    for n in (1, 3, 5, 7, 9):
        for (P, R, C) in ((2, 19, 23), (1, n, n), (3, 40, 37)):
            A = rng.random((P, R, C)) * 2 - 1
            K = rng.random((n, n)) * 2 - 1
            ref = _interior_n(A, K, lambda a, K: correlate2d(a, K, mode="valid"))
            if not np.allclose(convK(A, K), ref, rtol=0, atol=1e-13):
                return False
    return True


def pin_n_torch(convK) -> bool:
    """Eq. 1 at width 7 as torch's conv2d (cross-correlation), float64, CPU."""
    import torch

    rng = np.random.default_rng(32)
    A = rng.random((3, 31, 26)) * 2 - 1
    K = rng.random((7, 7)) * 2 - 1
    valid = torch.nn.functional.conv2d(torch.from_numpy(A)[:, None],
                                       torch.from_numpy(K)[None, None])[:, 0].numpy()
    ref = np.zeros_like(A)
    ref[:, 3:-3, 3:-3] = valid
    return bool(np.allclose(convK(A, K), ref, rtol=0, atol=1e-13))


def pin_n_bruteforce_tiny(convK) -> bool:
    """Pure-Python Eq. 1 for n in {1, 3, 7} and every H, W in 1..10."""
    rng = np.random.default_rng(33)
    for n in (1, 3, 7):
        r = n // 2
        K = (rng.random((n, n)) * 2 - 1).tolist()
        for R in range(1, 11):
            for C in range(1, 11):
                A = rng.random((1, R, C)) * 2 - 1
                a = A[0].tolist()
                ref = [[0.0] * C for _ in range(R)]
                if R >= n and C >= n:
                    for y in range(r, R - r):
                        for x in range(r, C - r):
                            ref[y][x] = sum(a[y + i - r][x + j - r] * K[i][j]
                                            for i in range(n) for j in range(n))
                if not np.allclose(convK(A, np.array(K))[0], np.array(ref), rtol=0, atol=1e-14):
                    return False
    return True


def pin_n_shift(convK) -> bool:
    """A kernel with one 1 at (a, b) moves A by (a - r, b - r): exact."""
    rng = np.random.default_rng(34)
    A = rng.random((1, 12, 15))
    for n in (3, 5):
        r = n // 2
        for a in range(n):
            for b in range(n):
                K = np.zeros((n, n))
                K[a, b] = 1.0
                ref = np.zeros_like(A)
                ref[0, r:12 - r, r:15 - r] = A[0, a:12 - n + 1 + a, b:15 - n + 1 + b]
                if not np.array_equal(convK(A, K), ref):
                    return False
    return True


def pin_n_delta(convK) -> bool:
    """A unit impulse gives the kernel turned by 180 degrees around it."""
    n, r = 9, 4
    K = np.arange(1.0, n * n + 1).reshape(n, n)
    A = np.zeros((1, 21, 23))
    A[0, 10, 11] = 1.0
    ref = np.zeros((21, 23))
    ref[10 - r:10 + r + 1, 11 - r:11 + r + 1] = K[::-1, ::-1]
    return bool(np.array_equal(convK(A, K)[0], ref))


def pin_n_constant(convK) -> bool:
    """A constant image c gives c * sum(K) on the interior, 0 on the r-border."""
    K = np.arange(-12.0, 13.0).reshape(5, 5) / 8.0 + 0.25
    A = np.full((2, 9, 12), 3.0)
    ref = np.zeros_like(A)
    ref[:, 2:-2, 2:-2] = 3.0 * K.sum()
    return bool(np.allclose(convK(A, K), ref, rtol=1e-15, atol=0))


CONV_N_PINS = {
    "scipy": pin_n_scipy,
    "torch": pin_n_torch,
    "bruteforce_tiny": pin_n_bruteforce_tiny,
    "shift": pin_n_shift,
    "delta": pin_n_delta,
    "constant": pin_n_constant,
}


def failing_n_pins(convK) -> list[str]:
    bad = []
    for name, pin in CONV_N_PINS.items():
        try:
            ok = pin(convK)
        except Exception:
            ok = False
        if not ok:
            bad.append(name)
    return bad


# ---- pins for one pyramid level (blur + 2x decimation) -----------------
# Each takes ``pyr(A, k) -> out``; out[p, yo, xo] is Eq. 1 at source pixel
# (2 yo, 2 xo), with the zero frame, for yo < ceil(R/2), xo < ceil(C/2).

def pin_pyr_bruteforce_tiny(pyr) -> bool:
    """Pure-Python sums at the even source pixels, every H, W in 1..11."""
    rng = np.random.default_rng(41)
    k = (rng.random(5) * 2 - 1).tolist()
    for R in range(1, 12):
        for C in range(1, 12):
            A = rng.random((1, R, C)) * 2 - 1
            a = A[0].tolist()
            Ro, Co = (R + 1) // 2, (C + 1) // 2
            ref = [[0.0] * Co for _ in range(Ro)]
            for yo in range(Ro):
                for xo in range(Co):
                    y, x = 2 * yo, 2 * xo
                    if 2 <= y < R - 2 and 2 <= x < C - 2:
                        ref[yo][xo] = sum(a[y + i - 2][x + j - 2] * k[i] * k[j]
                                          for i in range(5) for j in range(5))
            got = pyr(A, k)
            if got.shape != (1, Ro, Co) or not np.allclose(got[0], np.array(ref), rtol=0,
                                                           atol=1e-14):
                return False
    return True


def pin_pyr_constant(pyr) -> bool:
    """Constant c: c (sum k)^2 where the source pixel is interior, else 0."""
    k = np.array([0.5, -0.25, 1.0, 0.125, 0.75])
    A = np.full((2, 13, 10), 3.0)
    got = pyr(A, k)
    ref = np.zeros((2, 7, 5))
    for yo in range(7):
        for xo in range(5):
            if 2 <= 2 * yo < 11 and 2 <= 2 * xo < 8:
                ref[:, yo, xo] = 3.0 * k.sum() ** 2
    return got.shape == ref.shape and bool(np.allclose(got, ref, rtol=1e-15, atol=0))


def pin_pyr_ramp(pyr) -> bool:
    """A = a + b y + c x: at source (2 yo, 2 xo) the closed form of the conv5
    ramp pin, so a half-pixel shift of the sampling grid fails."""
    k = np.array([0.05, 0.1, 0.15, 0.3, 0.4])
    a, b, c = 0.5, 2.0, -3.0
    R, C = 15, 18
    yy, xx = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    A = (a + b * yy + c * xx)[None].astype(np.float64)
    S = k.sum()
    m = float(np.dot(np.arange(-2, 3), k))
    full = np.zeros((R, C))
    full[2:-2, 2:-2] = (S * S * (a + b * yy + c * xx) + S * m * (b + c))[2:-2, 2:-2]
    got = pyr(A, k)
    return bool(np.allclose(got[0], full[::2, ::2], rtol=1e-13, atol=1e-13))


PYR_PINS = {
    "bruteforce_tiny": pin_pyr_bruteforce_tiny,
    "constant": pin_pyr_constant,
    "ramp": pin_pyr_ramp,
}


def failing_pyr_pins(pyr) -> list[str]:
    bad = []
    for name, pin in PYR_PINS.items():
        try:
            ok = pin(pyr)
        except Exception:
            ok = False
        if not ok:
            bad.append(name)
    return bad


# ---- rounding / decoding pins -------------------------------------------

def _bf16_table():
    bits = np.arange(1 << 16, dtype=np.uint32)
    with np.errstate(invalid="ignore"):      # the NaN patterns widen quietly
        vals = (bits << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return bits.astype(np.uint16), vals


def nearest_even_bf16(x: float) -> int:
    """Brute force: the bf16 pattern nearest to the finite double x, compared
    with exact rationals; ties go to the even pattern (fraction LSB 0)."""
    bits, vals = _bf16_table()
    same = (np.signbit(vals) == np.signbit(x)) & np.isfinite(vals)
    cand = np.where(same)[0]
    v = vals[cand]
    order = np.argsort(np.abs(v - x), kind="stable")[:4]
    fx = Fraction(x)
    best = min(order, key=lambda i: (abs(Fraction(float(v[i])) - fx),
                                     int(bits[cand[i]]) & 1))
    return int(bits[cand[best]])


# ---- two-pass form with a 16-bit intermediate ----------------------------------

T16_FORMATS = {"f16": (10, -14), "bf16": (7, -126)}  # fraction bits, min normal exponent


def _rne_py(x: float, mbits: int, emin: int) -> float:
    """RNE of a finite double to a binary format with `mbits` fraction bits,
    written independently of the oracle: the quantum at x's exponent (fixed
    below the smallest normal), then Python's round(), which sends halves to
    the even integer."""
    if x == 0.0:
        return 0.0
    _, e = math.frexp(abs(x))          # |x| = m 2^e, m in [0.5, 1)
    q = math.ldexp(1.0, max(e - 1, emin) - mbits)
    return math.copysign(round(abs(x) / q) * q, x)


def _brute_t16(a2d, k, mbits, emin):
    """Loops in the oracle's order: row pass on every row (taps left to right,
    from 0.0), each value rounded, column pass top to bottom."""
    R, C = a2d.shape
    out = np.zeros((R, C))
    if R < 5 or C < 5:
        return out
    T = np.zeros((R, C))
    for y in range(R):
        for x in range(2, C - 2):
            t = 0.0
            for b in range(5):
                t += float(a2d[y, x + b - 2]) * float(k[b])
            T[y, x] = _rne_py(t, mbits, emin)
    for y in range(2, R - 2):
        for x in range(2, C - 2):
            s = 0.0
            for a in range(5):
                s += float(T[y + a - 2, x]) * float(k[a])
            out[y, x] = s
    return out


def pin_t16_bruteforce_tiny(conv_t) -> bool:
    """Same operations in the same order as the brute force: equal exactly,
    for both formats, signed and unsigned data, values down to the binary16
    subnormal range, all sizes 1..9 (below 5: zeros)."""
    rng = np.random.default_rng(77)
    for fmt, (mb, em) in T16_FORMATS.items():
        for _ in range(24):
            R, C = (int(v) for v in rng.integers(1, 10, size=2))
            scale = float(rng.choice([1.0, 1e-6, 300.0]))
            A = (rng.random((2, R, C)) - float(rng.choice([0.0, 0.5]))) * scale
            k = rng.random(5) - float(rng.choice([0.0, 0.3]))
            got = conv_t(A, k, fmt)
            for p in range(2):
                if not np.array_equal(got[p], _brute_t16(A[p], k, mb, em)):
                    return False
    return True


def pin_t16_exact_dyadic(conv_t) -> bool:
    """Pixels 0..3 with taps [1,4,6,4,1]/16: every intermediate is an integer
    over 16 below 4, exact in both formats, so the result is Eq. 1 exactly."""
    rng = np.random.default_rng(78)
    A = rng.integers(0, 4, size=(3, 23, 31)).astype(np.float64)
    k = np.array([1, 4, 6, 4, 1]) / 16.0
    ref = _eq1(A, k)
    return all(np.array_equal(conv_t(A, k, f), ref) for f in T16_FORMATS)


def _eq1(A, k):
    """Eq. 1 with K = k k^T on the interior, 25 shifted products in FP64."""
    P, R, C = A.shape
    B = np.zeros_like(A)
    for a in range(5):
        for b in range(5):
            B[:, 2:R - 2, 2:C - 2] += k[a] * k[b] * A[:, a:R - 4 + a, b:C - 4 + b]
    return B


def pin_t16_error_bound(conv_t) -> bool:
    """Against Eq. 1 in FP64: each intermediate carries a relative error of at
    most 2^-(mbits+1), so |B_t - B| <= 2^-(mbits+1) sum_a |k_a| |T_a| (+ FP64
    noise), and random data does show a nonzero difference."""
    rng = np.random.default_rng(79)
    A = rng.random((2, 40, 37))
    k = rng.random(5)
    k /= k.sum()
    P, R, C = A.shape
    T = np.zeros_like(A)
    for b in range(5):
        T[:, :, 2:C - 2] += k[b] * A[:, :, b:C - 4 + b]
    mag = np.zeros_like(A)
    for a in range(5):
        mag[:, 2:R - 2, :] += abs(k[a]) * np.abs(T[:, a:R - 4 + a, :])
    mag[:, :, :2] = 0
    mag[:, :, C - 2:] = 0
    ref = _eq1(A, k)
    for f, (mb, _) in T16_FORMATS.items():
        d = np.abs(conv_t(A, k, f) - ref)
        if not np.all(d <= 2.0 ** -(mb + 1) * mag * (1 + 1e-12) + 1e-15):
            return False
        if not np.any(d > 0):
            return False
    return True


T16_PINS = {
    "t16_bruteforce_tiny": pin_t16_bruteforce_tiny,
    "t16_exact_dyadic": pin_t16_exact_dyadic,
    "t16_error_bound": pin_t16_error_bound,
}


def failing_t16_pins(conv_t) -> list[str]:
    bad = []
    for name, pin in T16_PINS.items():
        try:
            ok = pin(conv_t)
        except Exception:
            ok = False
        if not ok:
            bad.append(name)
    return bad
