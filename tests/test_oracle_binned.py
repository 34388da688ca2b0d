"""Pins of the oracle's bin-integrated ("binned") profiles, Table tab:profile.

The binned value of a profile at grid point nu_k is its mean over the bin
[nu_k - dnu/2, nu_k + dnu/2].  Pins, none of which reuse the oracle's method:
* the Gauss-Legendre rule against numpy's and against exact polynomial moments;
* binned Gaussian and Lorentzian against erf and atan differences in 50-digit
  mpmath arithmetic (far wings included, where the plain differences cancel);
* binned Voigt against the Voigt profile as a convolution, the Gaussian
  average of the Lorentzian's exact bin integral, integrated by mpmath;
* the Gaussian (gamma -> 0) and Lorentzian (alpha -> 0) limits of the Voigt;
* the refinement identity of bin means (a bin's mean is the average of its
  two halves' means), which a midpoint or wrongly scaled formula fails;
* the small-bin limit fbar = f + dnu^2 f''/24 + O(dnu^4);
* sums over consecutive bins telescoping to the exact mass between the outer
  edges, and the same for sigma of a few lines (Eq. xsec with the cut-off rule).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import synth

LN2 = math.log(2.0)
KINDS = [(4, "doppler"), (6, "lorentz"), (7, "voigt")]


def test_gauss_legendre_rule(orc):
    x, w = orc.gl_rule()
    xr, wr = np.polynomial.legendre.leggauss(16)
    np.testing.assert_allclose(np.sort(x), np.sort(xr), rtol=0, atol=2e-16)
    np.testing.assert_allclose(w[np.argsort(x)], wr[np.argsort(xr)], rtol=1e-14)
    for k in range(32):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert float(np.sum(w * x ** k)) == pytest.approx(exact, abs=2e-15)


def _mp_gauss_bin(d, dnu, alpha):
    with mp.workdps(50):
        X = mp.sqrt(mp.log(2)) / mp.mpf(alpha)
        a = (mp.mpf(d) - mp.mpf(dnu) / 2) * X
        b = (mp.mpf(d) + mp.mpf(dnu) / 2) * X
        return float((mp.erf(b) - mp.erf(a)) / (2 * mp.mpf(dnu)))


def _mp_lorentz_bin(d, dnu, gamma):
    with mp.workdps(50):
        a = (mp.mpf(d) - mp.mpf(dnu) / 2) / mp.mpf(gamma)
        b = (mp.mpf(d) + mp.mpf(dnu) / 2) / mp.mpf(gamma)
        return float((mp.atan(b) - mp.atan(a)) / (mp.pi * mp.mpf(dnu)))


def _mp_voigt_bin(d, dnu, alpha, gamma):
    # V = G * L: the bin integral of V is the Gaussian average of the exact
    # bin integral of the Lorentzian centred at s, (atan((d_b - s)/gamma) -
    # atan((d_a - s)/gamma)) / pi.
    with mp.workdps(30):
        sg = mp.mpf(alpha) / mp.sqrt(2 * mp.log(2))
        g = mp.mpf(gamma)
        da, db = mp.mpf(d) - mp.mpf(dnu) / 2, mp.mpf(d) + mp.mpf(dnu) / 2

        def f(s):
            return mp.exp(-s * s / (2 * sg * sg)) * (mp.atan((db - s) / g) - mp.atan((da - s) / g))

        pts = sorted({-mp.inf, mp.mpf(0), da, db, mp.inf})
        # finer breakpoints around the Gaussian core and the bin edges
        extra = [k * sg for k in (-8, -4, -2, -1, 1, 2, 4, 8)] + [da - 3 * g, da + 3 * g, db - 3 * g, db + 3 * g]
        pts = sorted(set(pts) | set(extra))
        val = mp.quad(f, pts)
        return float(val / (mp.pi * sg * mp.sqrt(2 * mp.pi) * mp.mpf(dnu)))


@pytest.mark.parametrize("alpha,dnu", [(0.013, 0.01), (0.1, 0.05), (1e-4, 0.01), (0.5, 0.001)])
def test_binned_gaussian_against_mpmath(orc, alpha, dnu):
    X = math.sqrt(LN2) / alpha
    h = X * dnu
    for xc in [0.0, 0.2, -0.7, 1.3, 3.0, -5.5, 9.0, 20.0]:
        d = xc / X
        ref = _mp_gauss_bin(d, dnu, alpha)
        got = orc.binned(orc.BIN_DOPPLER, d, dnu, alpha, 0.0)
        # the edges x -+ h/2 are rounded to FP64 (absolute error ~|x| eps); in
        # the wing a shift dx of an edge changes the bin mean by ~2|x| dx / h
        # relative, so narrow bins far out are this ill-conditioned
        tol = 2e-13 + 8e-16 * (abs(xc) + 1.0) ** 2 / h
        if ref > 1e-290:
            assert got == pytest.approx(ref, rel=tol, abs=0), (xc, alpha, dnu)
        assert orc.binned(orc.BIN_DOPPLER, -d, dnu, alpha, 0.0) == got


@pytest.mark.parametrize("gamma,dnu", [(0.02, 0.01), (1e-4, 0.01), (3.0, 0.05), (0.05, 0.5)])
def test_binned_lorentz_against_mpmath(orc, gamma, dnu):
    for d in [0.0, 0.003, -0.011, 0.02, 0.25, -3.0, 25.0, 1.0e3]:
        ref = _mp_lorentz_bin(d, dnu, gamma)
        got = orc.binned(orc.BIN_LORENTZ, d, dnu, 0.0, gamma)
        assert got == pytest.approx(ref, rel=2e-14, abs=0), (d, gamma, dnu)


@pytest.mark.parametrize("d,dnu,alpha,gamma", [
    (0.0, 0.01, 0.029, 0.02),      # core, comparable widths
    (0.013, 0.01, 0.029, 0.02),
    (-0.2, 0.01, 0.029, 0.02),     # near wing
    (3.0, 0.01, 0.029, 0.02),      # far wing
    (0.0, 0.01, 1e-4, 1e-6),       # bin far wider than the profile
    (0.01, 0.01, 1e-4, 1e-6),      # next bin: Lorentzian wing only
    (0.004, 0.01, 0.05, 1e-6),     # Gaussian-dominated core
    (0.3, 0.01, 0.05, 1e-6),       # Gaussian-dominated, far
    (0.0, 0.05, 0.01, 2.0),        # Lorentzian-dominated
    (7.0, 0.05, 0.01, 2.0),
])
def test_binned_voigt_against_convolution(orc, d, dnu, alpha, gamma):
    ref = _mp_voigt_bin(d, dnu, alpha, gamma)
    got = orc.binned(orc.BIN_VOIGT, d, dnu, alpha, gamma)
    assert got == pytest.approx(ref, rel=1e-12, abs=0)


def test_binned_voigt_limits(orc):
    dnu = 0.01
    for d in [0.0, 0.007, 0.04, 0.1]:
        g = orc.binned(orc.BIN_DOPPLER, d, dnu, 0.02, 0.0)
        assert orc.binned(orc.BIN_VOIGT, d, dnu, 0.02, 0.0) == pytest.approx(g, rel=1e-13, abs=0)
        lor = orc.binned(orc.BIN_LORENTZ, d, dnu, 0.0, 0.03)
        assert orc.binned(orc.BIN_VOIGT, d, dnu, 1e-9, 0.03) == pytest.approx(lor, rel=1e-9, abs=0)


@pytest.mark.parametrize("kind,name", KINDS)
def test_refinement_identity(orc, kind, name):
    # mean over a bin = average of the means over its two halves
    rng = np.random.default_rng(3)
    for _ in range(40):
        dnu = 10.0 ** rng.uniform(-3, -1)
        alpha = 10.0 ** rng.uniform(-3.5, -1)
        gamma = 10.0 ** rng.uniform(-4, -1)
        d = rng.normal() * 5 * max(alpha, gamma, dnu)
        whole = orc.binned(kind, d, dnu, alpha, gamma)
        halves = 0.5 * (orc.binned(kind, d - dnu / 4, dnu / 2, alpha, gamma) +
                        orc.binned(kind, d + dnu / 4, dnu / 2, alpha, gamma))
        if whole > 1e-280:
            assert whole == pytest.approx(halves, rel=5e-13, abs=0), (name, d, dnu, alpha, gamma)


@pytest.mark.parametrize("kind,name", KINDS)
def test_small_bin_limit(orc, kind, name):
    # fbar - f = dnu^2 f''/24 + O(dnu^4): the difference falls 4x per halving
    alpha, gamma = 0.03, 0.02
    for d in [0.0, 0.017, 0.09]:
        f = orc.profile(kind - 4, d, alpha, gamma)
        e = [orc.binned(kind, d, h, alpha, gamma) - f for h in (1e-3, 5e-4, 2.5e-4)]
        assert e[0] / e[1] == pytest.approx(4.0, rel=2e-3)
        assert e[1] / e[2] == pytest.approx(4.0, rel=1e-3)


def test_bin_sums_telescope_to_exact_mass(orc):
    dnu = 0.01
    k = np.arange(-300, 301)
    # Gaussian: mass between the outer edges is erf(X e) at +-e
    alpha = 0.031
    s = math.fsum(orc.binned(orc.BIN_DOPPLER, float(x), dnu, alpha, 0.0) for x in k * dnu) * dnu
    e = 300.5 * dnu
    assert s == pytest.approx(math.erf(math.sqrt(LN2) * e / alpha), rel=1e-14)
    # Lorentzian: (2/pi) atan(e / gamma)
    gamma = 0.04
    s = math.fsum(orc.binned(orc.BIN_LORENTZ, float(x), dnu, 0.0, gamma) for x in k * dnu) * dnu
    assert s == pytest.approx(2.0 / math.pi * math.atan(e / gamma), rel=1e-14)
    # Voigt: the sum equals one bin over the whole span
    ks = np.arange(-40, 41)
    s = math.fsum(orc.binned(orc.BIN_VOIGT, float(x), dnu, 0.02, 0.01) for x in ks * dnu) * dnu
    big = orc.binned(orc.BIN_VOIGT, 0.0, 81 * dnu, 0.02, 0.01) * 81 * dnu
    assert s == pytest.approx(big, rel=1e-13)


def test_sigma_binned_mass_and_brute_force(orc):
    # Lines on a small grid: sum_k sigma_k dnu equals sum_i S_i times the exact
    # Lorentzian mass between the outer edges of line i's window; and sigma
    # equals the double loop over (line, bin) of S_i fbar_ik.
    wl = synth.workload("voigt_1e7", n_states=60, n_lines=12, nu_hi=20.0, seed=4, profile=synth.BIN_LORENTZ,
                      conditions=[synth.Condition(2000.0, 1.0, 2.0)])
    ln = wl.lines()
    cond = wl.conditions[0]
    r = orc.run_condition(wl, ln, cond)
    g = wl.grid
    nuk = g.nu0 + np.arange(g.n_bins) * g.dnu
    mass = 0.0
    brute = np.zeros(g.n_bins)
    for i in range(ln.n):
        if not r.nu[i] > 0:
            continue
        m = np.abs(nuk - r.nu[i]) <= cond.cutoff
        if not m.any():
            continue
        ks = np.nonzero(m)[0]
        lo = nuk[ks[0]] - g.dnu / 2 - r.nu[i]
        hi = nuk[ks[-1]] + g.dnu / 2 - r.nu[i]
        mass += r.S[i] * (math.atan(hi / r.gamma[i]) - math.atan(lo / r.gamma[i])) / math.pi
        for k in ks:
            brute[k] += r.S[i] * _mp_lorentz_bin(nuk[k] - r.nu[i], g.dnu, r.gamma[i])
    assert math.fsum(r.sigma) * g.dnu == pytest.approx(mass, rel=1e-12)
    m = brute > 1e-6 * brute.max()
    np.testing.assert_allclose(r.sigma[m], brute[m], rtol=1e-12)
