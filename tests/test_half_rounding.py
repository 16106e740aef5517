"""FP16 link stores round each real of the FP64 link once, to the nearest FP16
(ties to even).  Pinned by a brute-force search over every finite FP16 value,
on hand-picked doubles where rounding through FP32 first gives a different
FP16, for the oracle's definition (storage.round_links_r12) and for the method
the kernels use (round to odd in FP32, then to nearest in FP16), emulated here
step by step; the GPU tests check the kernels' stores bit for bit."""
import numpy as np
import pytest

from oracle import storage

# every finite FP16 value (as float64), with its bit pattern
_BITS = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
_VALS = _BITS.view(np.float16).astype(np.float64)
_FINITE = np.isfinite(_VALS)
_FV, _FB = _VALS[_FINITE], _BITS[_FINITE]


def nearest_half_bits(x):
    """Bits of the FP16 nearest to x by exhaustive search; ties go to the value
    with an even significand (last bit 0); beyond 65504 + half an ulp: Inf."""
    if np.isnan(x):
        return None
    if abs(x) >= 65520.0:
        return 0xFC00 if x < 0 else 0x7C00
    d = np.abs(_FV - x)
    best = d.min()
    cand = _FB[d == best]
    if x == 0.0:   # signed zero keeps its sign
        return 0x8000 if np.signbit(x) else 0x0000
    cand = [int(c) for c in cand if (int(c) & 0x8000) == (0x8000 if x < 0 else 0)] or [int(c) for c in cand]
    if len(cand) > 1:
        cand = [c for c in cand if (c & 1) == 0]
    assert len(cand) == 1
    return cand[0]


# Doubles whose FP16 rounding differs when the value goes through FP32 first.
DOUBLE_ROUNDING = [
    1.0 + 2.0 ** -11 + 2.0 ** -30,            # above the tie: 1 + 2^-10 (through FP32: a tie -> 1)
    -(0.5 + 2.0 ** -12 + 2.0 ** -40),          # same, negative, at half the magnitude
    0.75 + 2.0 ** -12 + 2.0 ** -40,           # just above the tie after 0.75: 0.75 + 2^-11 (through FP32: 0.75)
    2.0 ** -25 + 2.0 ** -60,                  # just above half the smallest subnormal: 2^-24 (through FP32: 0)
    2.0 ** -20 + 2.0 ** -25 + 2.0 ** -55,     # subnormal range, above a tie
]


@pytest.mark.parametrize("x", DOUBLE_ROUNDING)
def test_cases_really_differ_through_fp32(x):
    once = nearest_half_bits(x)
    twice = nearest_half_bits(float(np.float32(x)))
    assert once != twice


def test_oracle_links_round_once():
    vals = np.array(DOUBLE_ROUNDING + [0.3, -0.7071067811865476, 1.0, 0.0, 1e-9, 2.0 ** -14 * 1.5])
    n = len(vals)
    U = np.zeros((n, 3, 3), dtype=np.complex128)
    U[:, 0, 0] = vals + 1j * vals[::-1]
    U[:, 1, 2] = -vals + 0.5j * vals
    r = storage.round_links_r12(U, "f16")
    for a, b in [(0, 0), (1, 2)]:
        got = r[:, a, b]
        for k in range(n):
            for part, want_src in ((got[k].real, U[k, a, b].real), (got[k].imag, U[k, a, b].imag)):
                want = _VALS[nearest_half_bits(want_src)]
                assert part == want, (k, a, b, want_src, part, want)


def test_oracle_links_f32_round_once():
    # FP32 rows: numpy's complex128 -> complex64 conversion, nearest even
    x = 1.0 + 2.0 ** -24 + 2.0 ** -50   # above the FP32 tie
    U = np.zeros((1, 3, 3), dtype=np.complex128)
    U[0, 0, 1] = x
    r = storage.round_links_r12(U, np.complex64)
    assert r[0, 0, 1].real == 1.0 + 2.0 ** -23


def round_to_odd_then_half(xs):
    """The kernels' conversion, emulated step by step: FP64 -> FP32 toward zero
    (the nearest-even FP32, stepped back one ulp toward zero where it rounded
    away), the last FP32 bit set where that was inexact, then FP32 -> FP16 to
    nearest even."""
    xs = np.asarray(xs, dtype=np.float64)
    f = xs.astype(np.float32)
    away = np.abs(f.astype(np.float64)) > np.abs(xs)
    f = np.where(away, np.nextafter(f, np.float32(0)), f)
    inexact = f.astype(np.float64) != xs
    fb = f.view(np.uint32) | inexact.astype(np.uint32)
    with np.errstate(over="ignore"):   # beyond 65504: Inf, as intended
        return fb.view(np.float32).astype(np.float16).view(np.uint16)


def test_round_to_odd_method_hand_picked():
    xs = np.array(DOUBLE_ROUNDING + [-x for x in DOUBLE_ROUNDING]
                  + [0.0, -0.0, 65504.0, 65519.99, 65520.0, -1e9, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26,
                     2.0 ** -14, 2.0 ** -14 - 2.0 ** -25, 5e-324, 1.0, -0.5])
    got = round_to_odd_then_half(xs)
    for x, h in zip(xs, got):
        assert int(h) == nearest_half_bits(x), (x, hex(int(h)))


def test_round_to_odd_method_random():
    rng = np.random.default_rng(1401)
    # link-like values, plus values at, just above and just below FP16 ties in every binade
    xs = np.concatenate([rng.uniform(-1, 1, 4000),
                         rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 5, 2000)])
    e = rng.integers(-24, 15, 3000).astype(np.float64)
    m = rng.integers(0, 1 << 10, 3000).astype(np.float64)
    tie = (1.0 + (m + 0.5) / 1024.0) * 2.0 ** e
    xs = np.concatenate([xs, tie, np.nextafter(tie, np.inf), np.nextafter(tie, -np.inf), -tie])
    got = round_to_odd_then_half(xs)
    # numpy's float64 -> float16 cast rounds once, to nearest even: an independent check
    assert np.array_equal(got, xs.astype(np.float16).view(np.uint16))
    for x, h in zip(xs[::97], got[::97]):
        assert int(h) == nearest_half_bits(x)
    # and rounding through FP32 to nearest instead would not do
    twice = xs.astype(np.float32).astype(np.float16).view(np.uint16)
    assert np.count_nonzero(twice != got) > 0
