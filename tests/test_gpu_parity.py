"""GPU path vs oracle, element by element, through the C-ABI.

Tolerances (spec bar, written here): max relative error over grid
points with sigma_ref >= 1e-6 of the peak: 1e-10 for the FP64 form, 1e-4 for
the FP32 form; partition functions 1e-12; FP64 intensities 1e-12; FP32
intensities (S~ exp(s_b)) 1e-6.  Inputs: seeded synthetic workloads of
``synth`` at sizes the oracle finishes in seconds (several tiles, ragged
last tile, lines beyond both grid ends).
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, gpu_inputs, gpu_sigma, log, make_plan, oracle_sigma, rel_err, workload

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-10, FP32: 1e-4}


def _check_sigma(name, got, ref, prec, st=None):
    e, l1, n = rel_err(got, ref)
    log(f"[{name}] prec={'fp32' if prec else 'fp64'} max_rel={e:.3e} L1={l1:.3e} bins={n}"
        + (f" stats={st}" if st else ""))
    assert n > 0
    assert e <= TOL[prec], f"{name}: {e} > {TOL[prec]}"
    # bins the oracle leaves at exactly zero stay zero
    assert np.all(got[ref == 0.0] == 0.0)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_partition_functions(prec):
    import torch
    for k, kw in [("voigt_1e7", dict(n_states=200000, n_lines=10)),
                  ("twotemp_1e9", dict(n_states=200000, n_lines=10, n_chunks=1))]:
        wl = workload(k, **kw)
        plan = make_plan(wl, prec, 16)
        ds, _ = gpu_inputs(wl, wl.lines())
        Q, dQ = plan.partition_function(ds)
        torch.cuda.synchronize()
        Q, dQ = Q.cpu().numpy(), dQ.cpu().numpy()
        for c, cond in enumerate(wl.conditions):
            q, dq = oracle.partition(wl.states, wl.population, cond.T, cond.T_vib, cond.T_rot)
            assert Q[c] == pytest.approx(q, rel=1e-12, abs=0)
            if wl.population == 0:
                assert dQ[c] == pytest.approx(dq, rel=1e-12, abs=0)
            else:
                assert np.isnan(dQ[c])
        log(f"[Q] {k} Q={Q}")
        plan.close()


@pytest.mark.parametrize("k,prec", [("voigt_1e7", FP64), ("voigt_1e7", FP32),
                                    ("twotemp_1e9", FP64), ("twotemp_1e9", FP32)])
def test_line_intensities(k, prec):
    import torch
    kw = dict(n_states=50000, n_lines=200000) if k == "voigt_1e7" else dict(n_states=50000, n_lines=200000, n_chunks=1)
    wl = workload(k, **kw)
    ln = wl.lines()
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    S, ls = plan.line_intensities(ds, dl)
    torch.cuda.synchronize()
    S = S.cpu().numpy().astype(np.float64)
    ls = ls.cpu().numpy()
    for c, cond in enumerate(wl.conditions):
        q, _ = oracle.partition(wl.states, wl.population, cond.T, cond.T_vib, cond.T_rot)
        _, Sref, keep = oracle.intensities(wl.states, ln, wl.mode, wl.population, cond.T, q,
                                           cond.T_vib, cond.T_rot)
        got = S[c] * (np.exp(ls[c]) if prec == FP32 else 1.0)
        tol = 1e-12 if prec == FP64 else 1e-6
        m = keep == 1
        if prec == FP32:  # entries below the FP32 range of the chunk's maximum flush to zero
            m &= np.abs(Sref) >= np.abs(Sref).max() * 1e-30
        err = np.max(np.abs(got[m] - Sref[m]) / np.abs(Sref[m]))
        log(f"[S] {k} cond{c} prec={prec} max_rel={err:.3e}")
        assert err <= tol
        assert np.all(got[keep == 0] == 0.0)
    plan.close()


SMALL = {
    "doppler": ("doppler_1e4", dict(n_lines=3000, nu_hi=1500.0)),
    "voigt": ("voigt_1e7", dict(n_states=20000, n_lines=20000, nu_hi=1200.0)),
    "voigt_lowP": ("voigt_1e7", dict(n_states=20000, n_lines=15000, nu_hi=1000.0, seed=1202)),
    "lorentz": ("voigt_1e7", dict(n_states=20000, n_lines=20000, nu_hi=1000.0, profile=synth.LORENTZ)),
    "em2T": ("twotemp_1e9", dict(n_states=20000, n_lines=30000, n_chunks=1, nu_hi=2000.0)),
}


def _wl(name):
    k, kw = SMALL[name]
    wl = workload(k, **kw)
    if name == "voigt_lowP":  # near-Doppler Voigt: y ~ 1e-6..1e-3 (the 48-condition grid's low-pressure corner)
        wl.conditions = [synth.Condition(300.0, 1e-4, 25.0)]
    return wl


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_sigma_gather_small(name, prec):
    wl = _wl(name)
    k, kw = SMALL[name]
    for ci in range(len(wl.conditions)):
        if name == "voigt_lowP":
            ref = oracle.run_condition(wl, wl.lines(), wl.conditions[ci]).sigma
        else:
            ref = oracle_sigma(k, kw, ci)
        got, st, dt = gpu_sigma(wl, wl.lines(), prec)
        _check_sigma(f"{name}/c{ci}", got[ci], ref, prec, st)


@pytest.mark.parametrize("hwhm", [0.002, 0.037, 0.3])
@pytest.mark.parametrize("tile", [256, 512, 1024])
def test_sigma_gaussian_fixed_hwhm(hwhm, tile):
    """Fixed-HWHM Gaussian at step 0.01: lines with a few nonzero points (one
    line per lane), about a hundred (FP32) or a few hundred (FP64) nonzero
    points (64 points per wave step), and more than a tile (whole-tile rows)."""
    wl = synth.workload("voigt_1e7", n_states=5000, n_lines=5000, nu_hi=600.0, profile=synth.GAUSSIAN)
    wl.hwhm_fixed = hwhm
    ref = oracle.run_condition(wl, wl.lines(), wl.conditions[0]).sigma
    for prec in (FP64, FP32):
        got, st, _ = gpu_sigma(wl, wl.lines(), prec,
                               config=dict(tile_bins=tile, bucket_bins=256, persistent=1, waves_per_cu=16))
        _check_sigma(f"gaussian_fixed hwhm={hwhm} tile={tile}", got[0], ref, prec, st)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_sigma_scatter_small(prec):
    wl = _wl("voigt")
    k, kw = SMALL["voigt"]
    ref = oracle_sigma(k, kw, 0)
    got, st, _ = gpu_sigma(wl, wl.lines(), prec, algo=1)
    _check_sigma("voigt/scatter", got[0], ref, prec, st)


def test_window_pair_count_matches_oracle():
    wl = _wl("voigt")
    r = oracle.run_condition(wl, wl.lines(), wl.conditions[0], with_sigma=False)
    tot, counts = oracle.window_counts(r.nu, wl.conditions[0].cutoff, wl.grid)
    _, st, _ = gpu_sigma(wl, wl.lines(), FP32)
    log(f"[pairs] gpu={st['window_pairs']} oracle={tot} kept={st['lines_kept']}")
    assert st["window_pairs"] == tot
    assert st["lines_kept"] == int(np.sum(counts > 0))


@pytest.mark.parametrize("algo", [0, 1])
def test_doppler_1e4_full_size_every_point(algo):
    """The small FP64 workload at its stated size: 2,000 states, 1e4 lines,
    LTE absorption at T = 1000 K, mass 18, Doppler profile, grid 0-10000
    cm^-1 step 0.01 (1,000,001 points), cut-off 25 cm^-1; the oracle at every
    point; FP64 (the workload's form) and FP32."""
    wl = synth.workload("doppler_1e4")
    ln = wl.lines()
    assert ln.n == 10_000 and wl.grid.n_bins == 1_000_001
    ref = oracle.run_condition(wl, ln, wl.conditions[0]).sigma
    for prec in (FP64, FP32):
        got, st, _ = gpu_sigma(wl, ln, prec, algo=algo)
        _check_sigma(f"doppler_1e4 full algo={algo}", got[0], ref, prec, st)
        assert st["lines_in"] == 10_000


def _tie_workload(profile):
    """Lines whose wavenumbers lie exactly the cut-off away from points of an
    exactly representable grid (0, 0.25, ..., 25; cut-off 2): nu = 10 (points
    8 and 12 are at exactly the cut-off), nu = 26.75 (beyond the grid end,
    its wing reaching 24.75 and 25), and lines with nu < 0 and nu = 0
    (discarded)."""
    states = synth.States(np.array([0.0, 10.0, 26.75, 3.0, 1.5]), np.array([1.0, 3.0, 5.0, 3.0, 1.0]))
    lines = synth.Lines(np.array([1, 2, 0, 4, 3], np.int32), np.array([0, 0, 1, 3, 3], np.int32),
                        np.array([1.0, 2.0, 1.0, 1.0, 1.0], np.float32),
                        np.full(5, 0.3, np.float32), np.full(5, 0.5, np.float32))
    wl = synth.workload("voigt_1e7", n_states=5, n_lines=5, nu_hi=25.0, profile=profile)
    wl.states = states
    wl.grid = synth.Grid(0.0, 0.25, 101)
    wl.conditions = [synth.Condition(1000.0, 1.0, 2.0)]
    wl.hwhm_fixed = 0.5
    return wl, lines


@pytest.mark.parametrize("profile", [synth.GAUSSIAN, synth.LORENTZ, synth.VOIGT, synth.BIN_LORENTZ])
@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("algo", [0, 1])
def test_cutoff_tie_is_inclusive(profile, prec, algo):
    """The cut-off rule |nu_k - nu_i| <= cut is inclusive (section "Spectral
    synthesis"): points exactly the cut-off away receive the line, the next
    ones do not; lines beyond the grid end reach it with their wings; lines
    with nu <= 0 are discarded.  The oracle pins the same case on its own."""
    wl, ln = _tie_workload(profile)
    ref = oracle.run_condition(wl, ln, wl.conditions[0]).sigma
    got, st, _ = gpu_sigma(wl, ln, prec, algo=algo)
    got = got[0]
    nuk = np.arange(wl.grid.n_bins) * 0.25
    k8, k12, k775, k1225 = (int(np.searchsorted(nuk, v)) for v in (8.0, 12.0, 7.75, 12.25))
    assert ref[k8] > 0 and ref[k12] > 0 and ref[k775] == 0 and ref[k1225] == 0
    assert got[k8] > 0 and got[k12] > 0, (got[k8], got[k12])
    assert got[k775] == 0 and got[k1225] == 0
    assert got[int(np.searchsorted(nuk, 24.75))] > 0 and got[-1] > 0
    np.testing.assert_array_equal(got == 0.0, ref == 0.0)
    _check_sigma(f"cut-off tie prof={profile} algo={algo}", got, ref, prec, st)
    assert st["lines_kept"] == 2 and st["window_pairs"] == 17 + 2
