"""Pins of the oracle's constants, partition functions and line intensities.

Q(T) follows Eq. (pf) and Eq. (Q nlte 2T); the intensities follow
Eqs. (abs intensity lte), (nlte ab 2T), (ems intensity lte), (nlte em 2T).
The pins are closed forms and relations that a dropped term, a wrong sign or
a wrong power would break: CODATA's c2, geometric-series and rigid-rotor
partition functions, exact factorisation of the two-temperature Q on a
product set of (v, J) states, Kirchhoff's law between the emission and
absorption intensities, the LTE limit of the two-temperature forms, and
finite differences for the T-derivatives used by the adjoint.
"""
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _codata():
    vals = {}
    with open(os.path.join(HERE, "golden", "codata2018.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_constants_codata2018(orc):
    ref = _codata()
    h, c, kb, amu, c2 = orc.constants()
    assert h == ref["h_erg_s"] and c == ref["c_cm_per_s"] and kb == ref["kB_erg_per_K"]
    assert amu == ref["amu_g"]
    # c2 = h c / k_B, CODATA 2018 lists 1.438 776 877 x 10^-2 m K.
    assert c2 == pytest.approx(ref["c2_cm_K"], abs=1e-9)
    assert orc.c2() == c2


def _states(E, g, v=None, evib=None):
    return synth.States(np.asarray(E, np.float64), np.asarray(g, np.float64),
                        None if v is None else np.asarray(v, np.int32),
                        None if evib is None else np.asarray(evib, np.float64))


def test_Q_geometric_ladder(orc):
    # Harmonic ladder E_v = w v (v = 0..N-1), g = 1:
    # Q = (1 - q^N) / (1 - q), q = exp(-c2 w / T).
    w, N = 1234.5, 40
    st = _states(w * np.arange(N), np.ones(N))
    c2 = orc.c2()
    for T in [100.0, 700.0, 3000.0, 20000.0]:
        q = math.exp(-c2 * w / T)
        Q, dQ = orc.partition(st, orc.LTE, T)
        assert Q == pytest.approx((1 - q ** N) / (1 - q), rel=1e-14, abs=0)
        # dQ/dT of the closed form
        dq = q * c2 * w / T ** 2
        dref = (-(N) * q ** (N - 1) * dq * (1 - q) + (1 - q ** N) * dq) / (1 - q) ** 2
        assert dQ == pytest.approx(dref, rel=1e-12, abs=0)


def test_Q_rigid_rotor_high_T(orc):
    # E = B J (J + 1), g = 2J + 1: Q = T/(c2 B) + 1/3 + c2 B / (15 T) + O(T^-2)
    B = 1.5
    J = np.arange(0, 3000)
    st = _states(B * J * (J + 1.0), 2 * J + 1.0)
    c2 = orc.c2()
    for T in [300.0, 1000.0, 3000.0]:
        Q, _ = orc.partition(st, orc.LTE, T)
        t = T / (c2 * B)
        approx = t + 1.0 / 3.0 + 1.0 / (15.0 * t) + 4.0 / (315.0 * t * t)
        assert Q == pytest.approx(approx, rel=1e-9, abs=0)


def test_Q_limits(orc):
    rng = np.random.default_rng(0)
    E = np.concatenate([[0.0], rng.uniform(100.0, 5000.0, 9)])
    g = np.concatenate([[3.0], rng.integers(1, 20, 9).astype(float)])
    st = _states(E, g)
    Q0, _ = orc.partition(st, orc.LTE, 1.0)         # T -> 0: ground state only
    assert Q0 == pytest.approx(3.0, rel=1e-15, abs=0)
    Qinf, _ = orc.partition(st, orc.LTE, 1e12)     # T -> inf: total degeneracy
    assert Qinf == pytest.approx(g.sum(), rel=1e-8, abs=0)


def test_Q_two_temperature_factorises(orc):
    # On the full product set {(v, J)} with E = Evib(v) + Erot(J), Eq. (Q nlte 2T)
    # factorises exactly: Q(Tv, Tr) = Q_vib(Tv) Q_rot(Tr).
    nv, nj = 7, 60
    evib = 2000.0 * np.arange(nv) - 10.0 * np.arange(nv) * (np.arange(nv) + 1)
    J = np.arange(nj)
    erot = 1.3 * J * (J + 1.0)
    V, JJ = np.meshgrid(np.arange(nv), J, indexing="ij")
    E = evib[V] + erot[JJ]
    g = (2 * JJ + 1.0)
    st = _states(E.ravel(), g.ravel(), V.ravel(), evib)
    c2 = orc.c2()
    for Tv, Tr in [(3000.0, 1500.0), (800.0, 2500.0), (2000.0, 2000.0)]:
        Q, _ = orc.partition(st, orc.NLTE_2T, 0.0, Tv, Tr)
        qv = np.exp(-c2 * evib / Tv).sum()
        qr = ((2 * J + 1.0) * np.exp(-c2 * erot / Tr)).sum()
        assert Q == pytest.approx(qv * qr, rel=1e-13, abs=0)
    # equal temperatures reduce to LTE
    Q2, _ = orc.partition(st, orc.NLTE_2T, 0.0, 1700.0, 1700.0)
    Q1, _ = orc.partition(st, orc.LTE, 1700.0)
    assert Q2 == pytest.approx(Q1, rel=1e-13, abs=0)


def test_dQdT_finite_difference(orc):
    wl = synth.workload("doppler_1e4", n_states=500)
    for T in [300.0, 1000.0, 4000.0]:
        Q, dQ = orc.partition(wl.states, orc.LTE, T)
        h = 1e-4 * T
        fd = (orc.partition(wl.states, orc.LTE, T + h)[0] - orc.partition(wl.states, orc.LTE, T - h)[0]) / (2 * h)
        assert dQ == pytest.approx(fd, rel=1e-7, abs=0)


def _few_lines(n_states=300, n_lines=400, seed=5):
    wl = synth.workload("voigt_1e7", n_states=n_states, n_lines=n_lines, seed=seed)
    return wl, wl.lines()


def test_kirchhoff_emission_over_absorption(orc):
    # From the LTE absorption and emission formulas, for every line
    # eps_i / I_i = 2 h c^2 nu^3 / (exp(c2 nu / T) - 1)  (Kirchhoff / Planck).
    wl, ln = _few_lines()
    h, c, kb, _, c2 = orc.constants()
    for T in [300.0, 2000.0, 9000.0]:
        Q, _ = orc.partition(wl.states, orc.LTE, T)
        nu, Ia, keep = orc.intensities(wl.states, ln, orc.ABSORPTION, orc.LTE, T, Q)
        _, Ie, _ = orc.intensities(wl.states, ln, orc.EMISSION, orc.LTE, T, Q)
        m = (keep == 1) & (Ia > 1e-290) & (Ie > 1e-290)
        assert m.sum() > 100
        ratio = Ie[m] / Ia[m]
        ref = 2 * h * c * c * nu[m] ** 3 / np.expm1(c2 * nu[m] / T)
        np.testing.assert_allclose(ratio, ref, rtol=1e-12)


def test_two_temperature_equal_T_is_lte(orc):
    wl = synth.workload("twotemp_1e9", n_states=2000, n_lines=500, n_chunks=1)
    ln = wl.lines()
    for mode in (orc.ABSORPTION, orc.EMISSION):
        T = 2345.0
        Q1, _ = orc.partition(wl.states, orc.LTE, T)
        Q2, _ = orc.partition(wl.states, orc.NLTE_2T, 0.0, T, T)
        _, S1, _ = orc.intensities(wl.states, ln, mode, orc.LTE, T, Q1)
        _, S2, _ = orc.intensities(wl.states, ln, mode, orc.NLTE_2T, 0.0, Q2, T, T)
        np.testing.assert_allclose(S2, S1, rtol=1e-12)


def test_two_temperature_vibrational_scaling(orc):
    # Emission, Eq. (nlte em 2T): at fixed T_rot, changing T_vib multiplies each
    # line by exp(-c2 E_u,vib (1/Tv' - 1/Tv)) times the ratio of partition functions.
    wl = synth.workload("twotemp_1e9", n_states=2000, n_lines=500, n_chunks=1)
    ln = wl.lines()
    c2 = orc.c2()
    Tr, Tv1, Tv2 = 1500.0, 3000.0, 6000.0
    Qa, _ = orc.partition(wl.states, orc.NLTE_2T, 0.0, Tv1, Tr)
    Qb, _ = orc.partition(wl.states, orc.NLTE_2T, 0.0, Tv2, Tr)
    _, Sa, keep = orc.intensities(wl.states, ln, orc.EMISSION, orc.NLTE_2T, 0.0, Qa, Tv1, Tr)
    _, Sb, _ = orc.intensities(wl.states, ln, orc.EMISSION, orc.NLTE_2T, 0.0, Qb, Tv2, Tr)
    ev = wl.states.e_vib[wl.states.v[ln.upper]]
    m = keep == 1
    ref = Sa[m] * np.exp(-c2 * ev[m] * (1 / Tv2 - 1 / Tv1)) * Qa / Qb
    np.testing.assert_allclose(Sb[m], ref, rtol=1e-12)


def test_intensity_linear_in_A_and_dropped_lines(orc):
    wl, ln = _few_lines()
    T = 1500.0
    Q, _ = orc.partition(wl.states, orc.LTE, T)
    nu, S, keep = orc.intensities(wl.states, ln, orc.ABSORPTION, orc.LTE, T, Q)
    ln2 = synth.Lines(ln.upper, ln.lower, (ln.einstein_a * np.float32(2.0)).astype(np.float32))
    _, S2, _ = orc.intensities(wl.states, ln2, orc.ABSORPTION, orc.LTE, T, Q)
    np.testing.assert_allclose(S2, 2 * S, rtol=1e-15)
    # swapping upper and lower gives nu <= 0: the line is discarded
    ln3 = synth.Lines(ln.lower, ln.upper, ln.einstein_a)
    _, S3, k3 = orc.intensities(wl.states, ln3, orc.ABSORPTION, orc.LTE, T, Q)
    assert (k3 == 0).all() and (S3 == 0).all()


def test_ground_state_absorption_low_T_limit(orc):
    # A line from the ground state (E_l = 0, g_l = 1 only populated state as T -> 0):
    # I -> g_u A / (8 pi c nu^2) / g_l  (stimulated term -> 1, Q -> g_l).
    st = _states([0.0, 2000.0, 2500.0], [1.0, 5.0, 9.0])
    ln = synth.Lines(np.array([1], np.int32), np.array([0], np.int32), np.array([3.0], np.float32))
    _, c, _, _, _ = orc.constants()
    T = 20.0
    Q, _ = orc.partition(st, orc.LTE, T)
    _, S, _ = orc.intensities(st, ln, orc.ABSORPTION, orc.LTE, T, Q)
    assert S[0] == pytest.approx(5.0 * 3.0 / (8 * math.pi * c * 2000.0 ** 2), rel=1e-14, abs=0)


def test_log_scale_multiplies(orc):
    wl, ln = _few_lines()
    T = 1500.0
    Q, _ = orc.partition(wl.states, orc.LTE, T)
    s = np.random.default_rng(1).normal(size=ln.n).astype(np.float32)
    _, S, _ = orc.intensities(wl.states, ln, orc.ABSORPTION, orc.LTE, T, Q)
    _, Ss, _ = orc.intensities(wl.states, ln, orc.ABSORPTION, orc.LTE, T, Q, log_scale=s)
    np.testing.assert_allclose(Ss, S * np.exp(s.astype(np.float64)), rtol=1e-14)


@pytest.mark.parametrize("mode", [0, 1])
def test_dlnS_dT_finite_difference(orc, mode):
    wl, ln = _few_lines()
    T = 1800.0
    h = 1e-4 * T
    Q, dQ = orc.partition(wl.states, orc.LTE, T)
    d = orc.dlnS_dT(wl.states, ln, mode, T, Q, dQ)
    Qp, _ = orc.partition(wl.states, orc.LTE, T + h)
    Qm, _ = orc.partition(wl.states, orc.LTE, T - h)
    _, Sp, keep = orc.intensities(wl.states, ln, mode, orc.LTE, T + h, Qp)
    _, Sm, _ = orc.intensities(wl.states, ln, mode, orc.LTE, T - h, Qm)
    m = (keep == 1) & (Sp > 1e-280) & (Sm > 1e-280)
    fd = (np.log(Sp[m]) - np.log(Sm[m])) / (2 * h)
    np.testing.assert_allclose(d[m], fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())
