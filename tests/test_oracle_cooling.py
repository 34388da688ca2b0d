"""Pins of the oracle's cooling function, Eq. (cf).

W(T) = 1/(4 pi Q(T)) sum A h c nu g_u exp(-c2 E_u / T).  Pins:
* a harmonic ladder (E_v = w v, g = 1, one line v -> v-1 per level with
  A_v = v A_1, the harmonic-oscillator scaling): W = h c w A_1 <v> / (4 pi)
  with the closed form <v> = 1 / (exp(c2 w / T) - 1) (ladder long enough
  that its truncation is below rounding);
* a two-level system: W = A h c nu g_u e / (4 pi (g_l + g_u e)),
  e = exp(-c2 nu / T), and its high-temperature limit;
* W equals the sum of the LTE emission intensities, Eq. (ems intensity lte),
  which are pinned on their own (Kirchhoff, limits);
* lines with nu <= 0 add nothing.
"""
import math

import numpy as np
import pytest

import synth


def _consts(orc):
    h, c, kb, amu, c2 = orc.constants()
    return h, c, c2


def test_harmonic_ladder(orc):
    h, c, c2 = _consts(orc)
    w, A1, V = 1000.0, 3.0, 400
    st = synth.States(np.arange(V + 1) * w, np.ones(V + 1))
    v = np.arange(1, V + 1)
    ln = synth.Lines(v.astype(np.int32), (v - 1).astype(np.int32), (v * A1).astype(np.float32))
    T = np.array([50.0, 300.0, 1000.0, 2500.0, 5000.0])
    W, Q = orc.cooling(st, ln, T)
    vmean = 1.0 / np.expm1(c2 * w / T)
    np.testing.assert_allclose(W, h * c * w * A1 * vmean / (4 * math.pi), rtol=1e-13)
    np.testing.assert_allclose(Q, 1.0 / -np.expm1(-c2 * w / T), rtol=1e-14)


def test_two_level(orc):
    h, c, c2 = _consts(orc)
    nu, A, gl, gu = 1234.5, 7.0, 3.0, 5.0
    st = synth.States(np.array([0.0, nu]), np.array([gl, gu]))
    ln = synth.Lines(np.array([1], np.int32), np.array([0], np.int32), np.array([A], np.float32))
    T = np.array([10.0, 296.0, 3000.0, 1e7])
    W, _ = orc.cooling(st, ln, T)
    e = np.exp(-c2 * nu / T)
    ref = float(np.float32(A)) * h * c * nu * gu * e / (4 * math.pi * (gl + gu * e))
    np.testing.assert_allclose(W, ref, rtol=1e-14)
    hi = float(np.float32(A)) * h * c * nu * gu / (4 * math.pi * (gl + gu))
    assert W[-1] == pytest.approx(hi, rel=1e-5)


def test_equals_sum_of_emission_intensities(orc):
    wl = synth.workload("voigt_1e7", n_states=3000, n_lines=20000, nu_hi=20000.0, seed=31)
    ln = wl.lines()
    T = np.array([200.0, 1000.0, 4000.0])
    W, Q = orc.cooling(wl.states, ln, T)
    for j, t in enumerate(T):
        q, _ = orc.partition(wl.states, orc.LTE, t)
        assert Q[j] == pytest.approx(q, rel=1e-14, abs=0)
        _, S, keep = orc.intensities(wl.states, ln, orc.EMISSION, orc.LTE, t, q)
        assert W[j] == pytest.approx(math.fsum(S[keep == 1]), rel=1e-13, abs=0)


def test_nonpositive_wavenumbers_add_nothing(orc):
    st = synth.States(np.array([0.0, 100.0, 100.0]), np.array([1.0, 3.0, 3.0]))
    good = synth.Lines(np.array([1], np.int32), np.array([0], np.int32), np.array([2.0], np.float32))
    bad = synth.Lines(np.array([1, 0, 2], np.int32), np.array([0, 1, 1], np.int32),
                      np.array([2.0, 5.0, 9.0], np.float32))
    T = np.array([500.0])
    assert orc.cooling(st, bad, T)[0][0] == orc.cooling(st, good, T)[0][0]
