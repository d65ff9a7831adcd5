"""Pins of the oracle's storage rounding (``round_storage``), the reference
for every FP32 / FP16 parity test.

The reduced-precision forms compute in FP32 and store FP32 or FP16 with
round-to-nearest-even, FP16 subnormals kept (readings 23 and 24: an FP16
store rounds the FP32 result of the collision, so a value reaches FP16
through FP32).  The expected values below are fixed by IEEE 754 binary32 /
binary16 arithmetic, written as exact powers of two; none comes from the
oracle.  A rounding mode other than nearest-even fails the ties, a direct
FP64 -> FP16 conversion fails the double-rounding cases, and a flush of
subnormals fails the subnormal cases.
"""
import numpy as np
import pytest

import oracle as O

E = 2.0 ** -24   # FP16: smallest subnormal; FP32: half an ulp of 1
T = 2.0 ** -149  # FP32: smallest subnormal

F16_CASES = [
    (1 + 2.0 ** -11, 1.0),                          # tie -> even mantissa
    (1 + 3 * 2.0 ** -11, 1 + 2.0 ** -9),            # tie -> even (up)
    (1 + 2.0 ** -11 + 2.0 ** -22, 1 + 2.0 ** -10),  # above the tie, survives FP32
    (1 + 2.0 ** -11 + 2.0 ** -40, 1.0),             # FP32 drops 2^-40 first: tie -> 1
    (-(1 + 2.0 ** -11), -1.0),                      # symmetric
    (1e-6, 17 * E),                                 # g = 1e-6 scale: subnormal 16.78 E -> 17 E
    (2.5 * E, 2 * E),                               # subnormal tie -> even
    (3.5 * E, 4 * E),
    (0.5 * E, 0.0),                                 # half the smallest subnormal -> 0 (even)
    (0.75 * E, E),                                  # not flushed
    (0.5 * E + 2.0 ** -40, E),                      # FP32 keeps the excess -> rounds up
    (0.5 * E + 2.0 ** -50, 0.0),                    # FP32 drops it -> tie -> 0
    (2.0 ** -14 - E, 2.0 ** -14 - E),               # largest subnormal, exact
    (65519.0, 65504.0),                             # below the overflow threshold
    (65520.0, np.inf),                              # overflow threshold rounds to infinity
]

F32_CASES = [
    (1 + 2.0 ** -24, 1.0),                          # tie -> even
    (1 + 3 * 2.0 ** -24, 1 + 2.0 ** -22),           # tie -> even (up)
    (1 + 2.0 ** -24 + 2.0 ** -40, 1 + 2.0 ** -23),  # above the tie
    (-(1 + 3 * 2.0 ** -24), -(1 + 2.0 ** -22)),
    (1.5 * T, 2 * T),                               # subnormal tie -> even
    (2.5 * T, 2 * T),
    (0.5 * T, 0.0),
    (0.75 * T, T),                                  # subnormals not flushed
    (1e-6, 9.999999974752427e-07),                  # nearest binary32 to 1e-6
]


@pytest.mark.filterwarnings("ignore:overflow encountered in cast")
@pytest.mark.parametrize("storage", ["f16s"])
@pytest.mark.parametrize("x,want", F16_CASES)
def test_round_storage_f16(storage, x, want):
    got = O.round_storage(np.array([[x]]), storage)
    assert got.dtype == np.float64 and got[0, 0] == want


@pytest.mark.parametrize("storage", ["f32", "f32s"])
@pytest.mark.parametrize("x,want", F32_CASES)
def test_round_storage_f32(storage, x, want):
    got = O.round_storage(np.array([[x]]), storage)
    assert got.dtype == np.float64 and got[0, 0] == want


@pytest.mark.parametrize("storage", ["f64", "f64s"])
def test_round_storage_f64_is_identity(storage):
    x = np.array([[1 + 2.0 ** -52, 2.0 ** -1074, -0.1, 1e300]])
    got = O.round_storage(x, storage)
    assert np.array_equal(got, x) and got is not x


def test_round_storage_keeps_shape():
    x = np.linspace(-1, 1, 19 * 7).reshape(19, 7)
    for st in ("f64", "f32", "f32s", "f16s"):
        assert O.round_storage(x, st).shape == (19, 7)


# FP16 holding 2^12 x the value: the same IEEE roundings on a grid 12 binades lower
S12_CASES = [
    (2.0 ** -12 * (1 + 2.0 ** -11), 2.0 ** -12),               # tie -> even
    (2.0 ** -12 * (1 + 3 * 2.0 ** -11), 2.0 ** -12 * (1 + 2.0 ** -9)),
    (1e-6, 1074 * 2.0 ** -30),                                 # normal in the scaled form: 1073.74 -> 1074
    (2.0 ** -26, 2.0 ** -26),                                  # smallest normal of the scaled form
    (2.0 ** -36, 2.0 ** -36),                                  # smallest subnormal of the scaled form
    (0.75 * 2.0 ** -36, 2.0 ** -36),
    (-(1e-6), -(1074 * 2.0 ** -30)),
    (65504.0 / 4096, 65504.0 / 4096),                          # largest finite value: 15.99...
    (16.0, np.inf),                                            # 65536 overflows
]


@pytest.mark.filterwarnings("ignore:overflow encountered in cast")
@pytest.mark.parametrize("x,want", S12_CASES)
def test_round_storage_f16_scaled(x, want):
    got = O.round_storage(np.array([[x]]), "f16s12")
    assert got.dtype == np.float64 and got[0, 0] == want


def test_scaled_f16_is_f16_of_the_scaled_value():
    """On values whose scaled FP32 rounding is exact, the scaled form is the
    unscaled form of 4096 x the value, divided back."""
    x = np.array([[3.0e-5, -7.5e-7, 1.2e-3, 0.25]])
    assert np.array_equal(O.round_storage(x, "f16s12") * 4096.0,
                          O.round_storage(x * 4096.0, "f16s"))
