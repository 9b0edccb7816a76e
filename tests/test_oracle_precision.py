"""Pins of the storage rounding (no GPU): hand-worked BF16 / FP32 values, ties to even,
and a brute-force nearest-neighbour check."""
import numpy as np

from oracle import precision


def test_bf16_hand_values():
    # near 1 the BF16 spacing is 2^-7
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20,
                  -3.0, 0.0, 2.0 ** -126, 1.0 / 3.0])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -3.0, 0.0, 2.0 ** -126,
                     0.333984375])
    np.testing.assert_array_equal(precision.round_bf16(x), want)


def test_fp32_hand_values():
    x = np.array([1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, 0.1])
    want = np.array([1.0, 1 + 2.0 ** -22, 0.100000001490116119384765625])
    np.testing.assert_array_equal(precision.round_fp32(x), want)


def test_bf16_nearest_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(2000) * 10.0 ** rng.uniform(-6, 6, 2000)
    r = precision.round_bf16(x)
    for v, got in zip(x, r):
        e = np.floor(np.log2(abs(v)))
        ulp = 2.0 ** (e - 7)
        lo = np.floor(v / ulp) * ulp
        hi = lo + ulp
        best = lo if abs(v - lo) < abs(hi - v) else hi
        assert got == best or (abs(v - lo) == abs(hi - v))
        assert abs(got - v) <= 0.5 * ulp
