"""Pins of the oracle's adjoint: gradients of L = sum_k w_k (sigma_k - t_k)^2.

The oracle's analytic gradients with respect to T, P, gamma_ref, n_exp and the
per-line log-intensity scales are checked against central finite differences
of the oracle's own FP64 forward pass (a different computation: the forward
alone), and the per-line scale gradient against the dot-product identity
<J v, u> = <v, J^T u>, where J v is an exact forward pass because sigma is
linear in the intensities.
"""
import math

import numpy as np
import pytest

import synth


def _wl(prof, n_lines=60, seed=21):
    wl = synth.workload("voigt_1e7", n_states=300, n_lines=n_lines, nu_hi=30.0, seed=seed, profile=prof,
                      conditions=[synth.Condition(1900.0, 0.7, 4.0)])
    return wl, wl.lines()


def _loss(orc, wl, ln, cond, w, t, log_scale=None):
    r = orc.run_condition(wl, ln, cond, log_scale=log_scale)
    return math.fsum(w * (r.sigma - t) ** 2), r.sigma


def _perturb_lines(ln, gref=None, nexp=None):
    return synth.Lines(ln.upper, ln.lower, ln.einstein_a,
                       ln.gamma_ref if gref is None else gref.astype(np.float32),
                       ln.n_exp if nexp is None else nexp.astype(np.float32))


@pytest.mark.parametrize("prof", [0, 2, 3])
def test_adjoint_scalars_by_central_differences(orc, prof):
    wl, ln = _wl(prof)
    cond = wl.conditions[0]
    w = 10.0 ** np.random.default_rng(1).uniform(-2, 2, wl.grid.n_bins)
    # target: the forward at other conditions, so every bin has a residual
    tgt = orc.run_condition(wl, ln, synth.Condition(1700.0, 0.8, 4.0)).sigma
    L0, sig = _loss(orc, wl, ln, cond, w, tgt)
    g = 2.0 * w * (sig - tgt)
    adj = orc.adjoint(wl, ln, cond, g)
    # central differences converge as h^2 (at h = 1e-4 T the Doppler case is
    # still 5e-6 off); h = 1e-5 leaves ~5e-8 truncation and ~1e-11 rounding
    hT = 1e-5 * cond.T
    Lp, _ = _loss(orc, wl, ln, synth.Condition(cond.T + hT, cond.P, cond.cutoff), w, tgt)
    Lm, _ = _loss(orc, wl, ln, synth.Condition(cond.T - hT, cond.P, cond.cutoff), w, tgt)
    assert adj["dT"] == pytest.approx((Lp - Lm) / (2 * hT), rel=2e-6, abs=0)
    if prof != 0:
        hP = 1e-5 * cond.P
        Lp, _ = _loss(orc, wl, ln, synth.Condition(cond.T, cond.P + hP, cond.cutoff), w, tgt)
        Lm, _ = _loss(orc, wl, ln, synth.Condition(cond.T, cond.P - hP, cond.cutoff), w, tgt)
        assert adj["dP"] == pytest.approx((Lp - Lm) / (2 * hP), rel=2e-6, abs=0)
    else:
        assert adj["dP"] == 0.0


@pytest.mark.parametrize("prof", [2, 3])
def test_adjoint_per_line_directional(orc, prof):
    # Directional derivatives along Rademacher directions for gamma_ref and
    # n_exp (the perturbed values stay float32 exactly, so the forward sees them).
    wl, ln = _wl(prof)
    cond = wl.conditions[0]
    rng = np.random.default_rng(5)
    w = 10.0 ** rng.uniform(-2, 2, wl.grid.n_bins)
    tgt = orc.run_condition(wl, ln, synth.Condition(1700.0, 0.8, 4.0)).sigma
    _, sig = _loss(orc, wl, ln, cond, w, tgt)
    adj = orc.adjoint(wl, ln, cond, 2.0 * w * (sig - tgt))
    for _ in range(2):
        v = rng.choice([-1.0, 1.0], ln.n)
        gr = ln.gamma_ref.astype(np.float64)
        h = 2.0 ** -14
        gp = gr * (1 + h * v)
        gm = gr * (1 - h * v)
        Lp, _ = _loss(orc, wl, _perturb_lines(ln, gref=gp), cond, w, tgt)
        Lm, _ = _loss(orc, wl, _perturb_lines(ln, gref=gm), cond, w, tgt)
        dp = gp.astype(np.float32).astype(np.float64) - gm.astype(np.float32).astype(np.float64)
        fd = (Lp - Lm)
        assert float(np.dot(adj["d_gamma_ref"], dp)) == pytest.approx(fd, rel=1e-4, abs=0)
        ne = ln.n_exp.astype(np.float64)
        hn = 2.0 ** -12
        npl, nmi = ne + hn * v, ne - hn * v
        Lp, _ = _loss(orc, wl, _perturb_lines(ln, nexp=npl), cond, w, tgt)
        Lm, _ = _loss(orc, wl, _perturb_lines(ln, nexp=nmi), cond, w, tgt)
        dn = npl.astype(np.float32).astype(np.float64) - nmi.astype(np.float32).astype(np.float64)
        assert float(np.dot(adj["d_n_exp"], dn)) == pytest.approx(Lp - Lm, rel=1e-4, abs=0)


@pytest.mark.parametrize("prof", [0, 3])
def test_adjoint_log_scale_dot_product(orc, prof):
    wl, ln = _wl(prof, n_lines=80)
    cond = wl.conditions[0]
    rng = np.random.default_rng(8)
    u = rng.standard_normal(wl.grid.n_bins)         # cotangent
    v = rng.standard_normal(ln.n)                   # tangent in s
    r = orc.run_condition(wl, ln, cond)
    Jv = orc.sigma(r.nu, r.S * v, r.alpha, r.gamma, wl.profile, wl.grid, cond.cutoff)
    adj = orc.adjoint(wl, ln, cond, u)
    lhs = math.fsum(Jv * u)
    rhs = math.fsum(adj["d_log_scale"] * v)
    assert lhs == pytest.approx(rhs, rel=1e-12, abs=0)
    # and the per-line scale gradient by central differences of the forward
    s0 = np.zeros(ln.n, np.float32)
    i = int(np.argmax(np.abs(adj["d_log_scale"])))
    h = 2.0 ** -12
    sp = s0.copy(); sp[i] = h
    sm = s0.copy(); sm[i] = -h
    fp = orc.run_condition(wl, ln, cond, log_scale=sp).sigma
    fm = orc.run_condition(wl, ln, cond, log_scale=sm).sigma
    assert math.fsum((fp - fm) * u) / (2 * h) == pytest.approx(adj["d_log_scale"][i], rel=1e-6, abs=0)


@pytest.mark.parametrize("prof", [0, 2, 3])
def test_adjoint_bounds(orc, prof):
    """The per-line error scales (window sums of the terms' absolute values):
    with a positive cotangent the log-scale gradient's terms share one sign,
    so its scale equals the gradient; with a signed cotangent every scale
    bounds its gradient; the gamma sums agree with a brute-force sum over
    the window of |g| |df/dgamma| from central differences of the oracle's
    profile (a different computation)."""
    wl, ln = _wl(prof)
    cond = wl.conditions[0]
    rng = np.random.default_rng(7)
    g = rng.standard_normal(wl.grid.n_bins)
    pos = orc.adjoint(wl, ln, cond, np.abs(g))
    bpos = orc.adjoint_bounds(wl, ln, cond, np.abs(g))
    np.testing.assert_allclose(bpos["d_log_scale"], np.abs(pos["d_log_scale"]), rtol=1e-13, atol=0)
    ref = orc.adjoint(wl, ln, cond, g)
    b = orc.adjoint_bounds(wl, ln, cond, g)
    for k in ("d_log_scale", "d_gamma_ref", "d_n_exp"):
        assert np.all(b[k] >= np.abs(ref[k]) * (1 - 1e-12)), k
        assert np.all(b[k] <= bpos[k] * (1 + 1e-12)), k  # |g| is the same in both
    r = orc.run_condition(wl, ln, cond, with_sigma=False)
    _, _, Cabs = orc.adjoint_sums(r.nu, r.alpha, r.gamma, prof, wl.grid, cond.cutoff, g, absolute=True)
    if prof == 0:
        assert np.all(Cabs == 0.0)  # the Doppler profile has no Lorentzian width
        return
    nuk = wl.grid.nu0 + np.arange(wl.grid.n_bins) * wl.grid.dnu
    for i in np.flatnonzero(r.nu > 0)[:8]:
        m = np.abs(nuk - r.nu[i]) <= cond.cutoff
        h = 1e-6 * r.gamma[i]
        dfg = np.array([(orc.profile(prof, d, r.alpha[i], r.gamma[i] + h)
                         - orc.profile(prof, d, r.alpha[i], r.gamma[i] - h)) / (2 * h) for d in nuk[m] - r.nu[i]])
        brute = math.fsum(np.abs(g[m]) * np.abs(dfg))
        assert Cabs[i] == pytest.approx(brute, rel=1e-6, abs=0), i
