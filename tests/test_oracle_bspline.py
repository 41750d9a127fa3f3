"""Pins for the oracle's cardinal B-splines (O2) and moduli (O4).

The paper spreads each charge over the 4x4x4 surrounding points with cardinal
B-splines (section III.A.1) and interpolates forces with their derivatives
(section III.A.3).  The checks below fix the spline values by an independent
closed form (the truncated-power formula), published integer values,
partition of unity and symmetry, and the moduli by their closed forms.
"""
import json
import math
from fractions import Fraction
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))


def truncated_power_M(n, x):
    """Textbook explicit form M_n(x) = 1/(n-1)! sum_k (-1)^k C(n,k) (x-k)_+^(n-1),
    evaluated in exact rational arithmetic (it cancels badly in floating point)."""
    x = Fraction(x)
    s = Fraction(0)
    for k in range(n + 1):
        t = x - k
        if t > 0:
            s += (-1) ** k * math.comb(n, k) * t ** (n - 1)
    return float(s / math.factorial(n - 1))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8])
def test_M_matches_truncated_power_form(orc, n):
    for x in np.linspace(-0.5, n + 0.5, 57):
        assert orc.bspline_M(n, x) == pytest.approx(truncated_power_M(n, x), abs=1e-13)


@pytest.mark.parametrize("p", ["4", "6"])
def test_integer_values_are_eulerian(orc, p):
    vals = GOLD["bspline_integer_values"][p]
    den = GOLD["bspline_integer_values"]["denominator"][p]
    for k, v in enumerate(vals, start=1):
        assert orc.bspline_M(int(p), k) == pytest.approx(v / den, abs=1e-15)


def test_p4_closed_forms(orc):
    for w in np.linspace(0.0, 1.0, 11):
        th, _ = orc.bspline(4, w)
        expect = [(1 - w) ** 3 / 6, (3 * w ** 3 - 6 * w ** 2 + 4) / 6,
                  (-3 * w ** 3 + 3 * w ** 2 + 3 * w + 1) / 6, w ** 3 / 6]
        np.testing.assert_allclose(th, expect, atol=1e-15)


@pytest.mark.parametrize("p", [3, 4, 5, 6, 7, 8])
def test_partition_of_unity_symmetry_and_derivative(orc, p):
    rng = np.random.default_rng(p)
    for w in rng.uniform(0, 1, 25):
        th, dth = orc.bspline(p, w)
        assert th.sum() == pytest.approx(1.0, abs=1e-14)
        assert dth.sum() == pytest.approx(0.0, abs=1e-14)
        th_m, dth_m = orc.bspline(p, 1.0 - w)
        np.testing.assert_allclose(th, th_m[::-1], atol=1e-14)
        np.testing.assert_allclose(dth, -dth_m[::-1], atol=1e-13)
        h = 1e-6
        tp, _ = orc.bspline(p, w + h)
        tm, _ = orc.bspline(p, w - h)
        np.testing.assert_allclose(dth, (tp - tm) / (2 * h), atol=1e-8)


def test_first_moment_is_linear(orc):
    # sum_j theta_j * (point offset) reproduces the atom position: for points
    # g-p+1+j the centroid is g + w - p/2 (cardinal splines are centred).
    for p in (4, 6):
        for w in (0.0, 0.21, 0.5, 0.93):
            th, _ = orc.bspline(p, w)
            pts = np.arange(p) - p + 1
            assert (th * pts).sum() == pytest.approx(w - p / 2.0, abs=1e-13)


def test_moduli_closed_forms(orc):
    for K in (16, 32, 48, 64):
        m = np.arange(K)
        c = np.cos(2 * np.pi * m / K)
        b4 = orc.moduli(4, K)
        np.testing.assert_allclose(b4, 1.0 / (2.0 / 3.0 + c / 3.0) ** 2, rtol=1e-13)
        b6 = orc.moduli(6, K)
        c2 = np.cos(4 * np.pi * m / K)
        np.testing.assert_allclose(b6, 1.0 / ((66 + 52 * c + 2 * c2) / 120.0) ** 2, rtol=1e-13)
        for b in (b4, b6):
            assert b[0] == pytest.approx(1.0, abs=1e-14)
            np.testing.assert_allclose(b[1:], b[1:][::-1], rtol=1e-13)


def test_odd_order_moduli_closed_forms(orc):
    # For odd p the denominator sum_k M_p(k+1) exp(i k theta), theta = 2 pi m/K,
    # is exp(i (p-2) theta/2) times a real cosine polynomial: with the integer
    # values 1/2, 1/2 (p = 3) and 1/24, 11/24, 11/24, 1/24 (p = 5, checked
    # against the truncated-power form), |b(m)|^2 = 1/cos^2(theta/2) and
    # 1/((2 cos(3 theta/2) + 22 cos(theta/2))/24)^2.  Both vanish at the
    # Nyquist index m = K/2, the only entry left to the reading below.
    assert truncated_power_M(5, 1) == pytest.approx(1 / 24, abs=1e-15)
    assert truncated_power_M(5, 2) == pytest.approx(11 / 24, abs=1e-15)
    for K in (16, 32, 48):
        m = np.arange(K)
        th = 2 * np.pi * m / K
        reg = m != K // 2
        d3 = np.cos(th / 2) ** 2
        d5 = ((2 * np.cos(1.5 * th) + 22 * np.cos(th / 2)) / 24) ** 2
        np.testing.assert_allclose(orc.moduli(3, K)[reg], 1.0 / d3[reg], rtol=1e-12)
        np.testing.assert_allclose(orc.moduli(5, K)[reg], 1.0 / d5[reg], rtol=1e-12)


def test_odd_order_nyquist_is_finite(orc):
    # reading: the vanishing Nyquist denominator of an odd order takes the
    # mean of its two neighbours (the GPU path supports even orders only)
    b = orc.moduli(5, 32)
    assert np.all(np.isfinite(b))
    assert b[16] == pytest.approx(0.5 * (b[15] + b[17]))
