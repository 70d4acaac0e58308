"""The FP64 oracle against what the paper and the mathematics fix (CPU only)."""
import os

import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.txt")


@pytest.mark.parametrize("name", sorted(pins.CONV_PINS))
def test_direct_pins(name):
    assert pins.CONV_PINS[name](oracle.conv5), name


@pytest.mark.parametrize("name", ["scipy", "delta", "constant", "ramp",
                                  "exact_rational", "bruteforce_tiny"])
def test_twopass_pins(name):
    assert pins.CONV_PINS[name](oracle.conv5_twopass), name


def test_separability_fp64():
    """Two-pass FP64 == single-pass FP64 (Eq. 1 with K = k k^T) to rounding."""
    rng = np.random.default_rng(21)
    for shape in ((3, 64, 80), (1, 5, 5), (2, 7, 33)):
        A = rng.random(shape)
        k = rng.random(5) * 2 - 1
        d = oracle.conv5(A, k)
        t = oracle.conv5_twopass(A, k)
        scale = np.abs(A).max() * np.abs(k).sum() ** 2
        assert np.max(np.abs(d - t)) <= 1e-15 * 25 * scale


@pytest.mark.parametrize("name", sorted(pins.CONV_N_PINS))
def test_direct_n_pins(name):
    assert pins.CONV_N_PINS[name](oracle.conv_direct_n), name


def test_sep_n_width5_is_conv5():
    """Width n = 5 with K = k k^T is the width-5 form, term for term."""
    rng = np.random.default_rng(35)
    A = rng.random((3, 23, 31))
    k = rng.random(5) * 2 - 1
    assert np.array_equal(oracle.conv_sep_n(A, k), oracle.conv5(A, k))


def test_sep_n_factorises():
    """K = k k^T: the full-kernel sum equals a row pass then a column pass
    (written here with numpy sliding windows), to FP64 rounding."""
    rng = np.random.default_rng(36)
    for n in (1, 3, 7, 9):
        r = n // 2
        A = rng.random((2, 30, 27))
        k = rng.random(n) * 2 - 1
        win = np.lib.stride_tricks.sliding_window_view
        h = (win(A, n, axis=2) * k).sum(-1)            # [P, R, C - 2r]
        v = (win(h, n, axis=1) * k).sum(-1)            # [P, R - 2r, C - 2r]
        ref = np.zeros_like(A)
        ref[:, r:30 - r, r:27 - r] = v
        got = oracle.conv_sep_n(A, k)
        assert np.allclose(got, ref, rtol=0, atol=1e-13 * n * n)


def test_direct_n_rejects_even_width():
    with pytest.raises(ValueError):
        oracle.conv_direct_n(np.zeros((1, 8, 8)), np.zeros((4, 4)))


@pytest.mark.parametrize("name", sorted(pins.T16_PINS))
def test_twopass_t16_pins(name):
    assert pins.T16_PINS[name](oracle.conv5_twopass_t), name


def test_twopass_t_f32_is_twopass():
    rng = np.random.default_rng(37)
    A = rng.random((2, 19, 23))
    k = rng.random(5)
    assert np.array_equal(oracle.conv5_twopass_t(A, k, "f32"), oracle.conv5_twopass(A, k))


# plausible mistakes in the 16-bit intermediate, written around the FP64 forms:
# no rounding at all, the other 16-bit format, rounding only the rows the
# column pass writes, and truncation instead of round-to-nearest-even
def _t16_from(T_fn):
    """Row pass, T_fn on the intermediate, column pass, in the oracle's order
    of operations (so the right T_fn reproduces it exactly)."""
    def conv_t(A, k, f):
        A = np.asarray(A, dtype=np.float64)
        P, R, C = A.shape
        B = np.zeros_like(A)
        if R < 5 or C < 5:
            return B
        T = np.zeros_like(A)
        for b in range(5):
            T[:, :, 2:C - 2] = T[:, :, 2:C - 2] + A[:, :, b:C - 4 + b] * k[b]
        T = T_fn(T, f)
        for a in range(5):
            B[:, 2:R - 2, 2:C - 2] = B[:, 2:R - 2, 2:C - 2] + T[:, a:R - 4 + a, 2:C - 2] * k[a]
        return B
    return conv_t


def _other(f):
    return "bf16" if f == "f16" else "f16"


def _rows_only(T, f):
    out = T.copy()
    out[:, 2:-2] = oracle.decode(oracle.round_to(T[:, 2:-2], f), f)
    return out


def _truncate(T, f):
    mb, emin = pins.T16_FORMATS[f]
    _, e = np.frexp(T)
    q = np.ldexp(1.0, np.maximum(e - 1, emin) - mb)
    return np.trunc(T / q) * q


T16_MUTANTS = {
    "no_rounding": _t16_from(lambda T, f: T),
    "other_format": _t16_from(lambda T, f: oracle.decode(oracle.round_to(T, _other(f)), _other(f))),
    "interior_rows_only": _t16_from(_rows_only),
    "truncated": _t16_from(_truncate),
}


@pytest.mark.parametrize("name", sorted(T16_MUTANTS))
def test_t16_pins_reject_mutant(name):
    assert pins.failing_t16_pins(T16_MUTANTS[name]), name


def test_t16_reference_form_passes():
    """The mutants' scaffold with the right rounding passes every pin, so the
    mutants fail for their mistake, not for the scaffold."""
    good = _t16_from(lambda T, f: oracle.decode(oracle.round_to(T, f), f))
    assert pins.failing_t16_pins(good) == []


@pytest.mark.parametrize("name", sorted(pins.PYR_PINS))
def test_pyr_pins(name):
    assert pins.PYR_PINS[name](oracle.pyr_down), name


# plausible mistakes in a decimating level: odd sampling grid, floor instead
# of ceil for the output size, sampling before blurring
PYR_MUTANTS = {
    "odd_grid": lambda A, k: oracle.conv5(A, k)[..., 1::2, 1::2],
    "floor_size": lambda A, k: oracle.conv5(A, k)[..., :np.asarray(A).shape[-2] // 2 * 2:2,
                                                  :np.asarray(A).shape[-1] // 2 * 2:2],
    "decimate_then_blur": lambda A, k: oracle.conv5(np.asarray(A)[..., ::2, ::2], k),
}


@pytest.mark.parametrize("name", sorted(PYR_MUTANTS))
def test_pyr_pins_reject_mutant(name):
    assert pins.failing_pyr_pins(PYR_MUTANTS[name]), name


def _read_golden():
    cases, lines = [], [ln.strip() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        _, name, r, c = lines[i].split()
        r, c = int(r), int(c)
        k = [float(v) for v in lines[i + 1].split()[1:]]
        A = np.array([[float(v) for v in lines[i + 2 + y].split()] for y in range(r)])
        assert lines[i + 2 + r] == "expect"
        E = np.array([[float(v) for v in lines[i + 3 + r + y].split()] for y in range(r)])
        cases.append((name, A, k, E))
        i += 3 + 2 * r
    return cases


def test_golden_worked_examples():
    cases = _read_golden()
    assert {c[0] for c in cases} == {"single_pixel", "impulse", "too_small"}
    for name, A, k, E in cases:
        assert np.array_equal(oracle.conv5(A, k), E), name
        assert np.array_equal(oracle.conv5_twopass(A, k), E), name


def test_border_zero_and_tiny():
    rng = np.random.default_rng(22)
    A = rng.random((3, 20, 30)) + 1.0
    B = oracle.conv5(A, rng.random(5) + 0.1)
    assert np.all(B[:, :2, :] == 0) and np.all(B[:, -2:, :] == 0)
    assert np.all(B[:, :, :2] == 0) and np.all(B[:, :, -2:] == 0)
    assert np.all(B[:, 2:-2, 2:-2] > 0)
    for shape in ((3, 4, 100), (3, 100, 4), (1, 1, 1), (2, 0, 7), (0, 5, 5)):
        A = rng.random(shape)
        B = oracle.conv5(A, [1, 2, 3, 4, 5])
        assert B.shape == A.shape and not np.any(B)


def test_threads_do_not_change_result():
    rng = np.random.default_rng(23)
    A = rng.random((3, 50, 61))
    k = rng.random(5)
    assert np.array_equal(oracle.conv5(A, k, nthreads=1), oracle.conv5(A, k, nthreads=4))


def test_thread_count_does_not_leak_between_calls():
    """A call's thread count applies to that call only: after serial calls
    (the wrappers' default) the OpenMP default is unchanged, and an
    nthreads=0 call takes the full default team."""
    default = oracle.max_threads()
    A = np.random.default_rng(24).random((2, 20, 20))
    k = np.full(5, 0.2)
    oracle.conv5(A, k)
    oracle.conv_direct_n(A, np.full((3, 3), 1.0 / 9))
    assert oracle.last_team() == 1
    assert oracle.max_threads() == default
    oracle.conv5(A, k, nthreads=0)
    assert oracle.last_team() == default
    oracle.conv5(A, k, nthreads=3)
    assert oracle.last_team() == 3 and oracle.max_threads() == default
    oracle.conv_direct_n(A, np.full((3, 3), 1.0 / 9), nthreads=0)
    assert oracle.last_team() == default


# ---- storage decoding and rounding ---------------------------------------

def test_decode_f16_all_patterns():
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    got = oracle.decode(bits, "f16")
    ref = bits.view(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.array_equal(np.signbit(got[~nan]), np.signbit(ref[~nan]))


def test_decode_bf16_all_patterns():
    bits = np.arange(1 << 16, dtype=np.uint32)
    got = oracle.decode(bits.astype(np.uint16), "bf16")
    with np.errstate(invalid="ignore"):      # the NaN patterns widen quietly
        ref = (bits << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])


def _rounding_probe_values(rng, lo_exp, hi_exp, n):
    mant = rng.random(n) + 1.0
    ex = rng.integers(lo_exp, hi_exp, size=n)
    v = np.ldexp(mant, ex) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return v


def test_round_f16_matches_numpy():
    """numpy's binary64 -> binary16 cast rounds once to nearest even."""
    rng = np.random.default_rng(24)
    v = _rounding_probe_values(rng, -30, 17, 200000)
    # exact midpoints between neighbouring halves, and points just off them
    h = rng.integers(0, 0x7bff, size=20000).astype(np.uint16)
    a = h.view(np.float16).astype(np.float64)
    b = (h + 1).astype(np.uint16).view(np.float16).astype(np.float64)
    mid = (a + b) / 2
    v = np.concatenate([v, mid, np.nextafter(mid, 0), np.nextafter(mid, np.inf),
                        [0.0, -0.0, 65504.0, 65519.99, 65520.0, 1e9, -1e9, 2.0 ** -25,
                         2.0 ** -25 * 1.0000001, 2.0 ** -26]])
    got = oracle.round_to(v, "f16")
    with np.errstate(over="ignore"):         # +-1e9 and 65520 round to infinity
        ref = v.astype(np.float16).view(np.uint16)
    assert np.array_equal(got, ref)


def test_round_bf16_matches_bruteforce():
    """Nearest bf16 by exhaustive search with exact rationals, ties to even."""
    rng = np.random.default_rng(25)
    bits = rng.integers(0, 0x7f7f, size=60).astype(np.uint32)
    lo = (bits << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    hi = ((bits + 1) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    mid = (lo + hi) / 2
    vals = np.concatenate([mid, np.nextafter(mid, 0), np.nextafter(mid, np.inf),
                           _rounding_probe_values(rng, -140, 120, 60),
                           [2.0 ** -134, 3 * 2.0 ** -135, 2.0 ** -135, 1.0, 1.00390625]])
    got = oracle.round_to(vals, "bf16")
    for v, g in zip(vals, got):
        assert int(g) == pins.nearest_even_bf16(float(v)), v


def test_round_bf16_overflow_and_specials():
    big = float(np.float32(3.3895314e38))  # largest finite bf16
    got = oracle.round_to(np.array([big, 3.4e38, -3.4e38, np.inf, np.nan, 0.0, -0.0]), "bf16")
    assert list(got[:4]) == [0x7f7f, 0x7f80, 0xff80, 0x7f80]
    assert (int(got[4]) & 0x7f80) == 0x7f80 and (int(got[4]) & 0x7f)
    assert list(got[5:]) == [0x0000, 0x8000]
