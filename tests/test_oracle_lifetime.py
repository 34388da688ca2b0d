"""Pins of the oracle's predissociation (lifetime) broadening.

Section "Spectral synthesis": the upper-state lifetime tau broadens the
Voigt profile.  Reading: the natural Lorentzian of a state that decays with
lifetime tau has energy FWHM hbar/tau; in wavenumbers that is
(hbar/tau)/(h c) = 1/(2 pi c tau), so HWHM 1/(4 pi c tau), and Lorentzians
convolve into a Lorentzian with the summed HWHM, so it adds to the pressure
width.  Pins: the width against hbar/tau from the CODATA golden constants;
additivity with the pressure width; stable states (tau = inf) and unusable
values (tau <= 0, NaN) add nothing; the convolution of two Lorentzians by
quadrature equals the Lorentzian of the summed width (the additivity the
reading rests on); sigma of a few lines against a double loop over scipy's
voigt_profile with the lifetime widths.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "codata2018.txt")


def _golden():
    d = {}
    for ln in open(GOLD):
        if ln.strip() and not ln.startswith("#"):
            k, v = ln.split()
            d[k] = float(v)
    return d


def _lines(n, up, lo):
    return synth.Lines(np.asarray(up, np.int32), np.asarray(lo, np.int32), np.ones(n, np.float32),
                       np.full(n, 0.05, np.float32), np.full(n, 0.5, np.float32))


def test_natural_width_from_hbar_over_tau(orc):
    g = _golden()
    hbar = g["h_erg_s"] / (2 * math.pi)
    tau = np.array([np.inf, 1e-12, 3.3e-11, 1e-10, 0.0, -1.0, np.nan])
    ln = _lines(7, range(7), [0] * 7)
    nu = np.full(7, 1000.0)
    _, gam0 = orc.widths(nu, ln, orc.VOIGT, 2000.0, 0.0, 30.0)
    assert np.all(gam0 == 0.0)   # P = 0: no pressure width
    _, gam = orc.widths(nu, ln, orc.VOIGT, 2000.0, 0.0, 30.0, lifetime=tau)
    for t, gw in zip(tau, gam):
        if t > 0 and math.isfinite(t):
            fwhm = (hbar / t) / (g["h_erg_s"] * g["c_cm_per_s"])   # energy width -> cm^-1
            assert gw == pytest.approx(fwhm / 2, rel=1e-15)
        else:
            assert gw == 0.0
    assert gam[1] == pytest.approx(5.308837458876145 / 2, rel=1e-12)  # 1 ps: 5.31 cm^-1 FWHM


def test_adds_to_pressure_width(orc):
    tau = np.array([2e-12, np.inf])
    ln = _lines(2, [0, 1], [1, 0])
    nu = np.array([1500.0, 2500.0])
    _, gp = orc.widths(nu, ln, orc.VOIGT, 1500.0, 3.0, 30.0)
    _, gt = orc.widths(nu, ln, orc.VOIGT, 1500.0, 3.0, 30.0, lifetime=tau)
    _, gl = orc.widths(nu, ln, orc.VOIGT, 1500.0, 0.0, 30.0, lifetime=tau)
    assert gt[0] == pytest.approx(gp[0] + gl[0], rel=1e-15)
    assert gt[1] == gp[1]


def test_lorentzians_convolve_to_summed_width():
    g1, g2 = 0.03, 0.11
    L = lambda x, g: g / (math.pi * (x * x + g * g))
    for x in [0.0, 0.05, 0.4, 3.0]:
        v, _ = integrate.quad(lambda s: L(s, g1) * L(x - s, g2), -np.inf, np.inf, epsabs=0, epsrel=1e-12,
                              limit=400, points=None)
        assert v == pytest.approx(L(x, g1 + g2), rel=1e-9)


def test_sigma_with_lifetimes_brute_force(orc):
    wl = synth.workload("voigt_1e7", n_states=60, n_lines=14, nu_hi=20.0, seed=9,
                      conditions=[synth.Condition(2000.0, 0.5, 5.0)])
    synth.with_lifetimes(wl, frac=0.5, seed=3)
    ln = wl.lines()
    cond = wl.conditions[0]
    r = orc.run_condition(wl, ln, cond)
    tau = wl.states.lifetime[ln.upper]
    assert np.isfinite(tau).sum() >= 3
    nuk = wl.grid.nu0 + np.arange(wl.grid.n_bins) * wl.grid.dnu
    ref = np.zeros(wl.grid.n_bins)
    c = orc.constants()[1]
    for i in range(ln.n):
        if not r.nu[i] > 0:
            continue
        gp = float(ln.gamma_ref[i]) * (296.0 / cond.T) ** float(ln.n_exp[i]) * cond.P
        gt = gp + (1.0 / (4 * math.pi * c * tau[i]) if np.isfinite(tau[i]) else 0.0)
        sg = r.alpha[i] / math.sqrt(2 * math.log(2))
        d = nuk - r.nu[i]
        m = np.abs(d) <= cond.cutoff
        ref[m] += r.S[i] * special.voigt_profile(d[m], sg, gt)
    m = ref > 1e-6 * ref.max()
    np.testing.assert_allclose(r.sigma[m], ref[m], rtol=5e-12)
