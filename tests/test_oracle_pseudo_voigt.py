"""Pins of the oracle's pseudo-Voigt profiles (Table tab:profile).

Thompson-Cox-Hastings and Olivero-Longbothum pseudo-Voigts (the paper names
the methods only; the formulas are the cited ones, in the oracle's header).
Pins against things other than the oracle:
* unit area, by adaptive quadrature;
* the Gaussian limit (gamma = 0) and the Lorentzian limit (alpha -> 0);
* the profile's FWHM (found numerically on the oracle's output) against the
  exact Voigt FWHM (root of scipy's voigt_profile): within 2.5e-4 for the
  Olivero-Longbothum width (published accuracy 0.02%), within 5e-3 for the
  Thompson-Cox-Hastings width;
* the shape against scipy's voigt_profile: within 1.4% of the peak over
  Lorentzian/Gaussian width ratios 1e-3..1e3 (the published accuracy of the
  pseudo-Voigt mixture is about 1%).
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize, special

LN2 = math.log(2.0)


def _fwhm(fn, peak, hi):
    return 2.0 * optimize.brentq(lambda x: fn(x) - peak / 2.0, 0.0, hi, xtol=1e-15, rtol=1e-15)


@pytest.mark.parametrize("kind", [8, 9])
def test_unit_area_and_limits(orc, kind):
    for alpha, gamma in [(0.02, 0.01), (0.01, 0.3), (0.5, 1e-3)]:
        v, _ = integrate.quad(lambda d: orc.profile(kind, d, alpha, gamma), -np.inf, np.inf,
                              epsabs=0, epsrel=1e-12, limit=500)
        assert v == pytest.approx(1.0, rel=1e-9)
    for d in [0.0, 0.013, 0.05]:
        g = orc.profile(orc.DOPPLER, d, 0.03, 0.0)
        assert orc.profile(kind, d, 0.03, 0.0) == pytest.approx(g, rel=1e-12, abs=0)
        # Olivero-Longbothum at fG = 0 gives f = (0.5346 + sqrt 0.2166) fL =
        # 1.000003 fL, its own error; Thompson-Cox-Hastings gives f = fL, eta = 1
        lor = orc.profile(orc.LORENTZ, d, 0.0, 0.04)
        tol = 1e-5 if kind == 9 else 1e-9
        assert orc.profile(kind, d, 1e-12, 0.04) == pytest.approx(lor, rel=tol, abs=0)


@pytest.mark.parametrize("kind,tol", [(9, 2.5e-4), (8, 5e-3)])
def test_width_against_exact_voigt(orc, kind, tol):
    worst = 0.0
    for lr in np.linspace(-3, 3, 25):
        alpha, gamma = 0.5, 0.5 * 10.0 ** lr
        sg = alpha / math.sqrt(2 * LN2)
        vpk = special.voigt_profile(0.0, sg, gamma)
        fv = _fwhm(lambda x: special.voigt_profile(x, sg, gamma), vpk, 4 * (alpha + gamma))
        ppk = orc.profile(kind, 0.0, alpha, gamma)
        fp = _fwhm(lambda x: orc.profile(kind, x, alpha, gamma), ppk, 4 * (alpha + gamma))
        worst = max(worst, abs(fp / fv - 1.0))
    assert worst <= tol


@pytest.mark.parametrize("kind", [8, 9])
def test_shape_against_voigt(orc, kind):
    worst = 0.0
    for lr in np.linspace(-3, 3, 13):
        alpha, gamma = 0.5, 0.5 * 10.0 ** lr
        sg = alpha / math.sqrt(2 * LN2)
        x = np.linspace(-12, 12, 1201) * max(alpha, gamma)
        V = special.voigt_profile(x, sg, gamma)
        P = np.array([orc.profile(kind, float(d), alpha, gamma) for d in x])
        worst = max(worst, float(np.max(np.abs(P - V)) / V.max()))
    assert 1e-3 < worst <= 0.014
