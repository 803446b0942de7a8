"""Pins of the oracle's rounding operator fl_h (binary16, round to nearest,
ties to even) against NumPy's independent float64 -> float16 conversion, and
of the power-of-two scale used by the low-precision solve (paper, eq. vdlow)."""
import numpy as np
import pytest


def _all_half_values():
    bits = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16)
    h = bits.view(np.float16)
    return h[np.isfinite(h)].astype(np.float64)


def test_half_values_are_fixed_points(orc):
    v = _all_half_values()
    out = orc.fl_h(v)
    assert np.array_equal(out.view(np.uint64), v.view(np.uint64))


def test_midpoints_and_neighbours_match_numpy(orc):
    v = np.unique(_all_half_values())
    mids = (v[:-1] + v[1:]) / 2               # exact in binary64
    cand = np.concatenate([mids, np.nextafter(mids, np.inf), np.nextafter(mids, -np.inf)])
    with np.errstate(over="ignore"):
        ref = cand.astype(np.float16).astype(np.float64)
    assert np.array_equal(orc.fl_h(cand), ref)


def test_random_and_extreme_values_match_numpy(orc):
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(100000) * 10.0 ** rng.integers(-9, 6, 100000),
        [0.0, -0.0, 6.0e-8, 5.9604644775390625e-08, 2.98e-8, 2.9802322387695312e-08,
         65504.0, 65519.99, 65520.0, -65520.0, 1e300, -1e-300, np.inf, -np.inf],
    ])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    out = orc.fl_h(x)
    assert np.array_equal(out, ref)
    assert np.signbit(orc.fl_h(np.array([-0.0])))[0]
    assert np.isnan(orc.fl_h(np.array([np.nan])))[0]


@pytest.mark.parametrize("m", [1.0, 0.75, 0.5, 3.0, 1e-300, 1e300, 5e-324, 123.456])
def test_pow2_ceil(orc, m):
    s = orc.pow2_ceil(m)
    mant, e = np.frexp(s)
    assert mant == 0.5                         # a power of two
    assert 0.5 < m / s <= 1.0
