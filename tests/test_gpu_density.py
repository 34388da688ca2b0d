"""Non-LTE with custom vibronic densities on the GPU against the oracle.

Eqs. (Q nlte Nvib), (nlte ab pop density), (nlte em pop density): the
two-temperature emission workload's states and lines (11 manifolds) with user
weights n_vib per manifold (one of them zero) in place of T_vib, at its four
T_rot values.  Q to 1e-12, FP64 intensities to 1e-12, FP32 (S~ exp(s_b)) to
1e-6, sigma to 1e-10 (FP64) and 1e-4 (FP32) on bins >= 1e-6 of the peak, for
absorption and emission, Doppler (widths at T_rot) and binned Doppler.
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, gpu_inputs, gpu_sigma, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


def _wl(mode, n_lines=20000, profile=None, nu_hi=1500.0):
    wl = synth.workload("twotemp_1e9", n_states=20000, n_lines=n_lines, n_chunks=1, nu_hi=nu_hi, profile=profile)
    synth.with_vib_densities(wl, seed=11)
    wl.states.n_vib[4] = 0.0  # an unpopulated manifold
    wl.mode = mode
    return wl


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("mode", [0, 1])
def test_density_Q_and_intensities(prec, mode):
    import torch
    wl = _wl(mode)
    ln = wl.lines()
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    Q, dQ = plan.partition_function(ds)
    S, ls = plan.line_intensities(ds, dl)
    torch.cuda.synchronize()
    Q, S, ls = Q.cpu().numpy(), S.cpu().numpy().astype(np.float64), ls.cpu().numpy()
    for c, cond in enumerate(wl.conditions):
        q, _ = oracle.partition(wl.states, wl.population, cond.T, cond.T_vib, cond.T_rot)
        assert Q[c] == pytest.approx(q, rel=1e-12, abs=0)
        _, Sref, keep = oracle.intensities(wl.states, ln, wl.mode, wl.population, cond.T, q,
                                           cond.T_vib, cond.T_rot)
        got = S[c] * (np.exp(ls[c]) if prec == FP32 else 1.0)
        m = Sref > 0
        if prec == FP32:
            m &= Sref >= Sref.max() * 1e-30
        err = float(np.max(np.abs(got[m] - Sref[m]) / Sref[m]))
        log(f"[density] mode={mode} prec={prec} Tr={cond.T_rot} Q={Q[c]:.6e} S max_rel={err:.2e} over {m.sum()}")
        assert err <= (1e-12 if prec == FP64 else 1e-6)
        assert np.all(got[Sref == 0.0] == 0.0)
        assert m.sum() > 1000


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("mode,profile", [(0, synth.DOPPLER), (1, synth.DOPPLER), (1, synth.BIN_DOPPLER)])
def test_density_sigma(prec, mode, profile):
    # dense lines on a short grid, so that many bins lie within the compared
    # range of the peak (intensities span many decades)
    wl = _wl(mode, n_lines=40000, profile=profile, nu_hi=3000.0)
    ln = wl.lines()
    got, st, _ = gpu_sigma(wl, ln, prec)
    for c, cond in enumerate(wl.conditions):
        ref = oracle.run_condition(wl, ln, cond).sigma
        e, l1, n = rel_err(got[c], ref)
        log(f"[density sigma] mode={mode} prof={profile} prec={prec} Tr={cond.T_rot}: max_rel={e:.2e} L1={l1:.2e} bins={n}")
        assert n > 100
        assert e <= (1e-10 if prec == FP64 else 1e-4)
        if prec == FP64:  # the FP64 form holds its bound much further down
            e9, _, n9 = rel_err(got[c], ref, thr=1e-9)
            assert e9 <= 1e-10 and n9 > n


def test_density_needs_weights():
    P = X()
    wl = _wl(1, n_lines=100)
    ln = wl.lines()
    plan = make_plan(wl, FP64, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    ds.n_vib = None
    with pytest.raises(P.XsecError) as ei:
        plan.partition_function(ds)
    assert ei.value.code == P.XS_EINVAL
    plan.close()
