"""Pins of the oracle's non-LTE populations with custom vibronic densities.

Eqs. (Nvib), (F nlte Nvib), (Q nlte Nvib), (nlte ab pop density) and
(nlte em pop density): each manifold v carries a user weight n_v, rotational
levels follow T_rot, and Q(T_rot) sums g n_v exp(-c2 E_rot / T_rot).  Pins:
* with n_v = exp(-c2 E_vib(v) / T) and T_rot = T the populations are the LTE
  Boltzmann populations, so Q and both intensities equal the LTE ones;
* with n_v = exp(-c2 E_vib(v) / T_vib) the populations are the two-temperature
  ones: Q and the emission intensities equal the two-temperature values, and
  the absorption intensities differ only by the stimulated-emission factor,
  (1 - exp(-c2 nu / T_rot)) against (1 - exp(-c2 (nu_vib/T_vib + nu_rot/T_rot)));
* the intensities do not change when every n_v is scaled (Q scales alike), so
  the normalisation sum n_v = 1 of Eq. (Nvib) is immaterial to S;
* a single populated manifold: only lines from (absorption) or to (emission)
  it have intensity, and Q sums that manifold's rotational levels only.
"""
import math

import numpy as np
import pytest

import synth


def _wl(n_states=400, n_lines=3000, seed=5):
    wl = synth.workload("twotemp_1e9", n_states=n_states, n_lines=n_lines, n_chunks=1, nu_hi=30000.0, seed=seed)
    return wl


def _run(orc, wl, ln, mode, pop, T, Tv, Tr):
    Q, _ = orc.partition(wl.states, pop, T, Tv, Tr)
    nu, S, keep = orc.intensities(wl.states, ln, mode, pop, T, Q, Tv, Tr)
    return Q, nu, S, keep


@pytest.mark.parametrize("mode", [0, 1])
def test_boltzmann_densities_give_lte(orc, mode):
    wl = _wl()
    ln = wl.lines()
    T = 2300.0
    c2 = orc.c2()
    wl.states.n_vib = np.exp(-c2 * wl.states.e_vib / T)
    Qd, _, Sd, _ = _run(orc, wl, ln, mode, orc.NLTE_DENSITY, 0.0, 0.0, T)
    Ql, _, Sl, _ = _run(orc, wl, ln, mode, orc.LTE, T, 0.0, 0.0)
    assert Qd == pytest.approx(Ql, rel=1e-13, abs=0)
    m = Sl > 0
    assert m.sum() > 1000
    np.testing.assert_allclose(Sd[m], Sl[m], rtol=1e-12)


def test_vibrational_temperature_densities_give_two_temperatures(orc):
    wl = _wl(seed=6)
    ln = wl.lines()
    Tv, Tr = 5200.0, 1300.0
    c2 = orc.c2()
    ev = wl.states.e_vib
    wl.states.n_vib = np.exp(-c2 * ev / Tv)
    # emission: identical
    Qd, _, Sd, _ = _run(orc, wl, ln, 1, orc.NLTE_DENSITY, 0.0, 0.0, Tr)
    Q2, _, S2, _ = _run(orc, wl, ln, 1, orc.NLTE_2T, 0.0, Tv, Tr)
    assert Qd == pytest.approx(Q2, rel=1e-13, abs=0)
    m = S2 > 0
    np.testing.assert_allclose(Sd[m], S2[m], rtol=1e-12)
    # absorption: only the stimulated-emission factor differs
    _, nu, Sd, keep = _run(orc, wl, ln, 0, orc.NLTE_DENSITY, 0.0, 0.0, Tr)
    _, _, S2, _ = _run(orc, wl, ln, 0, orc.NLTE_2T, 0.0, Tv, Tr)
    v = wl.states.v
    nuv = ev[v[ln.upper]] - ev[v[ln.lower]]
    nur = nu - nuv
    fd = -np.expm1(-c2 * nu / Tr)
    f2 = -np.expm1(-c2 * (nuv / Tv + nur / Tr))
    m = (keep == 1) & (np.abs(S2) > 0) & (np.abs(f2) > 1e-8)
    assert m.sum() > 1000
    np.testing.assert_allclose(Sd[m] / S2[m], fd[m] / f2[m], rtol=1e-11)


@pytest.mark.parametrize("mode", [0, 1])
def test_density_scale_invariance(orc, mode):
    wl = _wl(seed=7)
    ln = wl.lines()
    synth.with_vib_densities(wl, seed=3)
    Q1, _, S1, _ = _run(orc, wl, ln, mode, orc.NLTE_DENSITY, 0.0, 0.0, 1800.0)
    assert math.fsum(wl.states.n_vib) == pytest.approx(1.0, rel=1e-15)
    wl.states.n_vib = wl.states.n_vib * 37.0
    Q2, _, S2, _ = _run(orc, wl, ln, mode, orc.NLTE_DENSITY, 0.0, 0.0, 1800.0)
    assert Q2 == pytest.approx(37.0 * Q1, rel=1e-13, abs=0)
    np.testing.assert_allclose(S2, S1, rtol=1e-13)


@pytest.mark.parametrize("mode", [0, 1])
def test_single_manifold(orc, mode):
    wl = _wl(seed=8)
    ln = wl.lines()
    v0 = 3
    nv = np.zeros(wl.states.e_vib.shape[0])
    nv[v0] = 1.0
    wl.states.n_vib = nv
    Tr = 2500.0
    Q, _, S, keep = _run(orc, wl, ln, mode, orc.NLTE_DENSITY, 0.0, 0.0, Tr)
    st = wl.states
    inv = st.v == v0
    c2 = orc.c2()
    Qref = math.fsum(st.g_tot[inv] * np.exp(-c2 * (st.energy[inv] - st.e_vib[v0]) / Tr))
    assert Q == pytest.approx(Qref, rel=1e-13, abs=0)
    src = ln.lower if mode == 0 else ln.upper
    own = st.v[src] == v0
    assert np.all(S[~own] == 0.0)
    assert np.all(S[own & (keep == 1)] > 0.0)
