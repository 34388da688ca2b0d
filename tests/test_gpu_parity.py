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
    for k, kw in [(2, dict(n_states=200000, n_lines=10)), (5, dict(n_states=200000, n_lines=10, n_chunks=1))]:
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
        log(f"[Q] config{k} Q={Q}")
        plan.close()


@pytest.mark.parametrize("k,prec", [(2, FP64), (2, FP32), (5, FP64), (5, FP32)])
def test_line_intensities(k, prec):
    import torch
    kw = dict(n_states=50000, n_lines=200000) if k == 2 else dict(n_states=50000, n_lines=200000, n_chunks=1)
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
        log(f"[S] config{k} cond{c} prec={prec} max_rel={err:.3e}")
        assert err <= tol
        assert np.all(got[keep == 0] == 0.0)
    plan.close()


SMALL = {
    "doppler": (1, dict(n_lines=3000, nu_hi=1500.0)),
    "voigt": (2, dict(n_states=20000, n_lines=20000, nu_hi=1200.0)),
    "voigt_lowP": (2, dict(n_states=20000, n_lines=15000, nu_hi=1000.0, seed=1202)),
    "lorentz": (2, dict(n_states=20000, n_lines=20000, nu_hi=1000.0, profile=synth.LORENTZ)),
    "em2T": (5, dict(n_states=20000, n_lines=30000, n_chunks=1, nu_hi=2000.0)),
}


def _wl(name):
    k, kw = SMALL[name]
    wl = workload(k, **kw)
    if name == "voigt_lowP":  # near-Doppler Voigt: y ~ 1e-6..1e-3 (the C3 low-pressure corner)
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
    wl = synth.config(2, n_states=5000, n_lines=5000, nu_hi=600.0, profile=synth.GAUSSIAN)
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
