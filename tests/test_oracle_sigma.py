"""Pins of the oracle's cross section, Eq. (xsec) with the cut-off rule.

sigma_k = sum_i S_i f_i(nu_k - nu_i) over the lines with nu_i > 0 and
|nu_k - nu_i| <= cut.  Pins: a brute-force double loop over every (line, bin)
pair with scipy's voigt_profile as f; an isolated line reproducing S f; the
integral of sigma equal to sum S_i minus the exact cut-off loss; superposition
and permutation invariance; the inclusive window edge; discarded and
outside-the-grid lines; sampled bins equal to the full grid.
"""
import math

import numpy as np
import pytest
from scipy import special

import synth

LN2 = math.log(2.0)


def _small(prof=synth.VOIGT, n_lines=14, nu_hi=20.0, seed=9, P=1.0, T=2000.0, cut=5.0):
    wl = synth.workload("voigt_1e7", n_states=60, n_lines=n_lines, nu_hi=nu_hi, seed=seed, profile=prof,
                      conditions=[synth.Condition(T, P, cut)])
    if prof == synth.GAUSSIAN:
        wl.hwhm_fixed = 0.05
    return wl, wl.lines(), wl.conditions[0]


@pytest.mark.parametrize("prof,nu_hi", [(0, 20000.0), (1, 20.0), (2, 20.0), (3, 20.0), (3, 20000.0)])
def test_brute_force_against_scipy(orc, prof, nu_hi):
    # Every (line, bin) pair of the grid, the predicate as printed, and the
    # profile from scipy (voigt_profile) or its closed form.
    wl, ln, cond = _small(prof, nu_hi=nu_hi)
    r = orc.run_condition(wl, ln, cond)
    nu0, dnu, N = wl.grid.nu0, wl.grid.dnu, wl.grid.n_bins
    nuk = nu0 + np.arange(N) * dnu
    ref = np.zeros(N)
    for i in range(ln.n):
        if not r.nu[i] > 0:
            continue
        sg = r.alpha[i] / math.sqrt(2 * LN2)
        d = nuk - r.nu[i]
        m = np.abs(d) <= cond.cutoff
        if prof == 3:
            f = special.voigt_profile(d[m], sg, r.gamma[i])
        elif prof == 2:
            f = r.gamma[i] / math.pi / (d[m] * d[m] + r.gamma[i] ** 2)
        else:
            f = np.exp(-d[m] * d[m] / (2 * sg * sg)) / (sg * math.sqrt(2 * math.pi))
        ref[m] += r.S[i] * f
    m = ref > 1e-6 * ref.max()
    assert m.sum() > (20 if prof in (0, 1) else 300)
    np.testing.assert_allclose(r.sigma[m], ref[m], rtol=5e-12)
    assert (r.sigma[ref == 0.0] == 0.0).all()


def test_isolated_line_is_S_times_profile(orc):
    grid = synth.Grid(0.0, 0.01, 3001)
    nu = np.array([12.3456789])
    for prof, alpha, gamma in [(0, 0.03, 0.0), (2, 0.0, 0.05), (3, 0.02, 0.01)]:
        sig = orc.sigma(nu, np.array([2.5e-20]), np.array([alpha]), np.array([gamma]), prof, grid, 3.0)
        k = np.arange(grid.n_bins)
        d = (0.0 + k * 0.01) - nu[0]
        inw = np.abs(d) <= 3.0
        ref = np.array([2.5e-20 * orc.profile(prof, x, alpha, gamma) if w else 0.0 for x, w in zip(d, inw)])
        np.testing.assert_array_equal(sig, ref)


def test_integral_equals_sum_minus_cutoff_loss(orc):
    # Well-resolved Doppler lines far from the grid ends: the sampled integral
    # sum_k sigma_k dnu equals sum_i S_i (1 - erfc(cut sqrt(ln2) / alpha_i)).
    rng = np.random.default_rng(4)
    n = 40
    nu = rng.uniform(30.0, 70.0, n)
    S = 10.0 ** rng.uniform(-22, -19, n)
    alpha = rng.uniform(0.03, 0.08, n)
    gamma = np.zeros(n)
    grid = synth.Grid(0.0, 0.005, 20001)
    for cut in [0.1, 0.25, 5.0]:
        sig = orc.sigma(nu, S, alpha, gamma, 0, grid, cut)
        lhs = math.fsum(sig) * grid.dnu
        # the window holds the bins within cut; its sampled area is the
        # truncated Gaussian area up to the half-bin end corrections, so use
        # cut values on the bin lattice relative to each centre: compare with
        # the per-line sampled sums instead where the end effects matter.
        per = [math.fsum(orc.sigma(nu[i:i + 1], S[i:i + 1], alpha[i:i + 1], gamma[i:i + 1], 0, grid, cut)) * grid.dnu
               for i in range(n)]
        assert lhs == pytest.approx(math.fsum(per), rel=1e-14, abs=0)
        if cut >= 1.0:
            ref = math.fsum(S * (1.0 - special.erfc(cut * math.sqrt(LN2) / alpha)))
            assert lhs == pytest.approx(ref, rel=1e-12, abs=0)


def test_lorentz_integral_cutoff_loss(orc):
    # Lorentzian with gamma >> dnu: sum_k L dnu over |d| <= cut equals
    # (2/pi) atan(cut/gamma) up to the trapezoid end correction.
    grid = synth.Grid(0.0, 0.001, 60001)
    nu = np.array([30.0])
    gamma = 0.05
    for cut in [2.0, 10.0]:
        sig = orc.sigma(nu, np.array([1.0]), np.array([0.0]), np.array([gamma]), 2, grid, cut)
        s = math.fsum(sig) * grid.dnu
        end = gamma / math.pi / (cut * cut + gamma * gamma) * grid.dnu  # two half-weights
        assert s - end == pytest.approx(2 / math.pi * math.atan(cut / gamma), rel=1e-8, abs=0)


def test_superposition_and_permutation(orc):
    wl, ln, cond = _small(3, n_lines=200, nu_hi=30.0)
    r = orc.run_condition(wl, ln, cond)
    perm = np.random.default_rng(2).permutation(ln.n)
    rp = orc.sigma(r.nu[perm], r.S[perm], r.alpha[perm], r.gamma[perm], 3, wl.grid, cond.cutoff)
    np.testing.assert_array_equal(r.sigma, rp)  # sorted by (nu, index) before summing
    a = orc.sigma(r.nu[:90], r.S[:90], r.alpha[:90], r.gamma[:90], 3, wl.grid, cond.cutoff)
    b = orc.sigma(r.nu[90:], r.S[90:], r.alpha[90:], r.gamma[90:], 3, wl.grid, cond.cutoff)
    m = r.sigma > 1e-12 * r.sigma.max()
    np.testing.assert_allclose(a[m] + b[m], r.sigma[m], rtol=1e-13)


def test_window_edge_inclusive_and_dropped_lines(orc):
    grid = synth.Grid(0.0, 0.25, 101)   # exactly representable grid
    cut = 2.0
    nu = np.array([10.0, -3.0, 0.0, 24.75 + cut, -1.5])
    S = np.ones(5)
    alpha = np.full(5, 0.5)
    gamma = np.zeros(5)
    sig = orc.sigma(nu, S, alpha, gamma, 0, grid, cut)
    k = np.arange(grid.n_bins)
    nuk = k * 0.25
    # line 0: bins 8.0 and 12.0 are exactly cut away and are included
    ref = np.where(np.abs(nuk - 10.0) <= cut, np.array([orc.profile(0, x, 0.5, 0.0) for x in nuk - 10.0]), 0.0)
    # lines 1 and 2 (nu <= 0) are discarded; line 3 is outside the grid
    # (26.75 > 25.0) but its wing reaches bins 24.75..25.0; line 4 has nu < 0.
    ref += np.where(np.abs(nuk - 26.75) <= cut, np.array([orc.profile(0, x, 0.5, 0.0) for x in nuk - 26.75]), 0.0)
    np.testing.assert_allclose(sig, ref, rtol=1e-15, atol=0)
    assert sig[np.searchsorted(nuk, 8.0)] > 0 and sig[np.searchsorted(nuk, 12.0)] > 0
    assert sig[np.searchsorted(nuk, 24.75)] > 0
    tot, counts = orc.window_counts(nu, cut, grid)
    assert list(counts) == [17, 0, 0, 2, 0] and tot == 19


def test_sampled_bins_equal_full_grid(orc):
    wl, ln, cond = _small(3, n_lines=300, nu_hi=40.0)
    r = orc.run_condition(wl, ln, cond)
    bins = synth.sample_bins(wl.grid.n_bins, 257, 12)
    rs = orc.run_condition(wl, ln, cond, bins=bins)
    np.testing.assert_array_equal(rs.sigma, r.sigma[bins])
