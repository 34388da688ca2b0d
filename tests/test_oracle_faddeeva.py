"""Pins of the oracle's Faddeeva function w(z) = exp(-z^2) erfc(-iz).

The Voigt profile of the paper's profile table (SciPy Voigt / wofz Voigt) is
Re w(z) / (sg sqrt(2 pi)).  The oracle computes w by a modified trapezoidal
rule; these tests tie it to values fixed by independent means: mpmath's
arbitrary-precision erfc, the closed forms w(0) = 1, Re w(iy) = erfcx(y),
Re w(x) = exp(-x^2) and Im w(x) = 2 D(x) / sqrt(pi) (Dawson's integral) on the
real axis, and w'(z) = -2 z w(z) + 2 i / sqrt(pi).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special


def _w_mp(x, y, dps):
    with mp.workdps(dps):
        z = mp.mpc(x, y)
        w = mp.exp(-z * z) * mp.erfc(-1j * z)
        wp = -2 * z * w + 2j / mp.sqrt(mp.pi)
        return complex(w), complex(wp), complex(w + z * wp)


XS = [0.0, 1e-3, 0.05, 0.4, 1.0, 2.2, 3.7, 5.1, 6.6, 7.95, 10.0, 31.0, 300.0, 4.0e3, 2.0e6]
YS = [1e-6, 1e-4, 1e-2, 0.3, 1.0, 3.0, 7.8, 7.9, 40.0, 1e3, 1e6]


@pytest.mark.parametrize("y", YS)
def test_w_matches_mpmath_on_log_grid(orc, y):
    # Relative error of Re w, the part the Voigt profile uses, <= 1e-13 (FP64
    # oracle requirement); w' and G = w + z w' (adjoint) <= 1e-12.
    for x in XS + [-x for x in XS[1:5]]:
        dps = 40 if max(abs(x), y) < 1e3 else 90
        w, wp, G = _w_mp(x, y, dps)
        a = orc.faddeeva(x, y)
        b, c = orc.faddeeva_deriv(x, y)
        assert abs(a.real - w.real) <= 1e-13 * abs(w.real), (x, y, a, w)
        assert abs(a.imag - w.imag) <= 1e-13 * abs(w) , (x, y, a, w)
        assert abs(b - wp) <= 1e-12 * abs(wp), (x, y, b, wp)
        assert abs(c - G) <= 1e-12 * abs(G), (x, y, c, G)


def test_w_dense_near_real_axis(orc):
    # Small y near and between the quadrature nodes: Re w ~ exp(-x^2) + O(y).
    rng = np.random.default_rng(7)
    for x in np.concatenate([np.linspace(0, 9.0, 181), rng.uniform(0, 9, 60)]):
        for y in (1e-8, 1e-5, 3e-3):
            w, _, _ = _w_mp(float(x), y, 40)
            a = orc.faddeeva(float(x), y)
            assert abs(a.real - w.real) <= 1e-13 * abs(w.real), (x, y)


def test_w_special_values(orc):
    assert abs(orc.faddeeva(0.0, 0.0) - 1.0) < 1e-15
    for y in [1e-4, 0.1, 1.0, 5.0, 7.0, 50.0, 1e4]:
        assert orc.faddeeva(0.0, y).real == pytest.approx(special.erfcx(y), rel=1e-14, abs=0)
    for x in [0.1, 0.7, 2.0, 4.0, 8.0, 15.0]:
        a = orc.faddeeva(x, 0.0)
        assert a.real == pytest.approx(math.exp(-x * x), rel=1e-13, abs=1e-300)
        assert a.imag == pytest.approx(2.0 / math.sqrt(math.pi) * special.dawsn(x), rel=1e-13, abs=0)


def test_w_symmetry(orc):
    for x, y in [(0.3, 0.2), (2.5, 1e-3), (11.0, 4.0), (1e3, 0.5)]:
        a, b = orc.faddeeva(x, y), orc.faddeeva(-x, y)
        assert a.real == pytest.approx(b.real, rel=1e-15, abs=0)
        assert a.imag == pytest.approx(-b.imag, rel=1e-15, abs=0)


def test_w_matches_scipy_wofz(orc):
    rng = np.random.default_rng(3)
    x = 10.0 ** rng.uniform(-3, 4, 400)
    y = 10.0 ** rng.uniform(-5, 4, 400)
    ref = special.wofz(x + 1j * y)
    for xi, yi, r in zip(x, y, ref):
        a = orc.faddeeva(float(xi), float(yi))
        assert abs(a.real - r.real) <= 1e-12 * abs(r.real)
