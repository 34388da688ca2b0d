"""Pins of the oracle's unit-area line profiles (Table tab:profile) and widths.

Doppler/Gaussian, Lorentzian and SciPy-convention Voigt, normalised to unit
area as required under Eq. (xsec).  Pins: scipy.special.voigt_profile (the
paper's "SciPy Voigt" method itself), the half-maximum property of the HWHM,
the Gaussian and Lorentzian limits of the Voigt profile, the exact tail
integrals erfc and arctan for the truncated unit area, the standard Doppler
and pressure width laws, and finite differences for the width derivatives
used by the adjoint.
"""
import math

import numpy as np
import pytest
from scipy import special

LN2 = math.log(2.0)


def test_voigt_matches_scipy_voigt_profile(orc):
    rng = np.random.default_rng(11)
    for _ in range(400):
        alpha = 10.0 ** rng.uniform(-5, 0)
        gamma = 10.0 ** rng.uniform(-6, 1)
        d = rng.choice([-1, 1]) * 10.0 ** rng.uniform(-4, 2)
        sg = alpha / math.sqrt(2 * LN2)
        ref = special.voigt_profile(d, sg, gamma)
        v = orc.profile(orc.VOIGT, d, alpha, gamma)
        if ref > 1e-300:
            assert v == pytest.approx(ref, rel=2e-12, abs=0), (d, alpha, gamma)


def test_gaussian_half_maximum_and_scipy(orc):
    for alpha in [1e-4, 0.013, 0.2]:
        g0 = orc.profile(orc.DOPPLER, 0.0, alpha, 0.0)
        assert orc.profile(orc.DOPPLER, alpha, alpha, 0.0) == pytest.approx(g0 / 2, rel=1e-14, abs=0)
        assert orc.profile(orc.DOPPLER, -alpha, alpha, 0.0) == pytest.approx(g0 / 2, rel=1e-14, abs=0)
        sg = alpha / math.sqrt(2 * LN2)
        for d in [0.0, 0.3 * alpha, 2.7 * alpha]:
            ref = math.exp(-d * d / (2 * sg * sg)) / (sg * math.sqrt(2 * math.pi))
            assert orc.profile(orc.DOPPLER, d, alpha, 0.0) == pytest.approx(ref, rel=1e-14, abs=0)


def test_lorentz_half_maximum_and_cauchy(orc):
    for gamma in [1e-3, 0.05, 2.0]:
        l0 = orc.profile(orc.LORENTZ, 0.0, 0.0, gamma)
        assert l0 == pytest.approx(1.0 / (math.pi * gamma), rel=1e-15, abs=0)
        assert orc.profile(orc.LORENTZ, gamma, 0.0, gamma) == pytest.approx(l0 / 2, rel=1e-15, abs=0)


def test_voigt_limits(orc):
    alpha, d = 0.02, 0.013
    g = orc.profile(orc.DOPPLER, d, alpha, 0.0)
    assert orc.profile(orc.VOIGT, d, alpha, 0.0) == pytest.approx(g, rel=1e-13, abs=0)
    assert orc.profile(orc.VOIGT, d, alpha, 1e-12) == pytest.approx(g, rel=1e-8, abs=0)
    gamma = 0.03
    lor = orc.profile(orc.LORENTZ, d, 0.0, gamma)
    assert orc.profile(orc.VOIGT, d, 1e-9, gamma) == pytest.approx(lor, rel=1e-10, abs=0)
    # far wing: V -> gamma / (pi d^2)
    assert orc.profile(orc.VOIGT, 40.0, alpha, gamma) == pytest.approx(gamma / (math.pi * 1600.0), rel=1e-5, abs=0)


def _quad(orc, prof, alpha, gamma, cut):
    from scipy import integrate
    val, _ = integrate.quad(lambda x: orc.profile(prof, x, alpha, gamma), -cut, cut,
                            points=[0.0], limit=500, epsabs=1e-14, epsrel=1e-13)
    return val


def test_unit_area_with_exact_tails(orc):
    # Gaussian: the sampled sum over all bins is spectrally exact once
    # alpha >~ 3 dnu, so it reproduces the unit area to rounding.
    alpha, dnu = 0.05, 0.005
    k = np.arange(-400, 401)
    s = sum(orc.profile(orc.DOPPLER, float(x), alpha, 0.0) for x in k * dnu) * dnu
    assert s == pytest.approx(1.0, abs=1e-14)
    # Truncated areas: Gaussian 1 - erfc(cut sqrt(ln2) / alpha); Lorentzian
    # (2/pi) atan(cut / gamma); Voigt against scipy's voigt_profile integrated
    # by the same adaptive quadrature.
    for alpha, cut in [(0.05, 0.12), (0.01, 0.004)]:
        ref = 1.0 - special.erfc(cut * math.sqrt(LN2) / alpha)
        assert _quad(orc, orc.DOPPLER, alpha, 0.0, cut) == pytest.approx(ref, rel=1e-11, abs=0)
    for gamma, cut in [(0.05, 3.0), (0.2, 25.0)]:
        ref = 2 / math.pi * math.atan(cut / gamma)
        assert _quad(orc, orc.LORENTZ, 0.0, gamma, cut) == pytest.approx(ref, rel=1e-11, abs=0)
    from scipy import integrate
    for alpha, gamma, cut in [(0.04, 0.03, 1.0), (0.01, 0.002, 25.0)]:
        sg = alpha / math.sqrt(2 * LN2)
        ref, _ = integrate.quad(lambda x: special.voigt_profile(x, sg, gamma), -cut, cut,
                                points=[0.0], limit=500, epsabs=1e-14, epsrel=1e-13)
        assert _quad(orc, orc.VOIGT, alpha, gamma, cut) == pytest.approx(ref, rel=1e-10, abs=0)


def test_widths_laws(orc):
    import synth
    h, c, kb, amu, _ = orc.constants()
    nu = np.array([10.0, 1000.0, 20000.0])
    ln = synth.Lines(np.zeros(3, np.int32), np.zeros(3, np.int32), np.ones(3, np.float32),
                     np.array([0.05, 0.02, 0.1], np.float32), np.array([0.5, 0.75, 0.3], np.float32))
    T, P, M = 1234.0, 3.5, 30.0
    alpha, gamma = orc.widths(nu, ln, orc.VOIGT, T, P, M)
    # Doppler HWHM: the Gaussian of the Maxwell velocity distribution
    # (std sqrt(kT/m) in velocity) scaled by nu/c, times sqrt(2 ln 2).
    sg_ref = nu / c * np.sqrt(kb * T / (M * amu))
    np.testing.assert_allclose(alpha, sg_ref * math.sqrt(2 * LN2), rtol=1e-14)
    g_ref = ln.gamma_ref.astype(float) * (296.0 / T) ** ln.n_exp.astype(float) * P
    np.testing.assert_allclose(gamma, g_ref, rtol=1e-14)
    a2, _ = orc.widths(nu, ln, orc.GAUSSIAN, T, P, M, hwhm_fixed=0.07)
    assert (a2 == 0.07).all()


@pytest.mark.parametrize("prof", [0, 2, 3])
def test_profile_derivatives_finite_difference(orc, prof):
    # df/dsg and df/dgamma of the oracle's adjoint sums against central
    # differences of the profile itself (one line, one bin at a time).
    import synth
    grid = synth.Grid(0.0, 0.01, 2001)
    rng = np.random.default_rng(prof)
    for _ in range(25):
        nu = float(rng.uniform(5.0, 15.0))
        alpha = float(10 ** rng.uniform(-3, -1))
        gamma = float(10 ** rng.uniform(-3, -0.5))
        w = 4.0 * (alpha + (gamma if prof != 0 else 0.0)) / 0.01
        k = int(round(nu / 0.01 + rng.uniform(-w, w)))
        g = np.zeros(grid.n_bins)
        g[k] = 1.0
        A, B, C = orc.adjoint_sums(np.array([nu]), np.array([alpha]), np.array([gamma]), prof, grid, 25.0, g)
        d = k * 0.01 - nu
        f = orc.profile(prof, d, alpha, gamma)
        assert A[0] == pytest.approx(f, rel=1e-14, abs=0)
        sg = alpha / math.sqrt(2 * LN2)
        hs = 1e-5 * sg
        fs = (orc.profile(prof, d, (sg + hs) * math.sqrt(2 * LN2), gamma)
              - orc.profile(prof, d, (sg - hs) * math.sqrt(2 * LN2), gamma)) / (2 * hs)
        hg = 1e-5 * gamma
        fg = (orc.profile(prof, d, alpha, gamma + hg) - orc.profile(prof, d, alpha, gamma - hg)) / (2 * hg)
        scale_s = abs(f) / sg + 1e-300
        scale_g = abs(f) / gamma + 1e-300
        assert abs(B[0] - fs) <= 1e-6 * scale_s + 1e-7 * abs(fs)
        assert abs(C[0] - fg) <= 1e-6 * scale_g + 1e-7 * abs(fg)
