"""Thompson and Olivero pseudo-Voigt profiles on the GPU against the oracle.

The benchmark line list reduced to 0-300 cm^-1 at 2000 K / 1 bar, at
300 K / 1e-4 bar (near-Gaussian) and at 300 K / 100 bar (near-Lorentzian),
with predissociation widths on a third of the upper states in the first
case; gather and scatter, FP64 (1e-10) and FP32 (1e-4) on bins >= 1e-6 of
the peak.  Their adjoint is not provided (XS_EUNSUPPORTED).
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, gpu_inputs, gpu_sigma, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
CASES = {
    "mid": [synth.Condition(2000.0, 1.0, 25.0)],
    "lowP": [synth.Condition(300.0, 1e-4, 25.0)],
    "highP": [synth.Condition(300.0, 100.0, 100.0)],
}


def _wl(kind, case):
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=3000, nu_hi=300.0, profile=kind, seed=1241,
                      conditions=CASES[case])
    if case == "mid":
        synth.with_lifetimes(wl, frac=0.33, seed=9)
    return wl


@pytest.mark.parametrize("kind", [synth.PV_THOMPSON, synth.PV_OLIVERO])
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("algo", [0, 1])
def test_pseudo_voigt_sigma(kind, case, prec, algo):
    wl = _wl(kind, case)
    ln = wl.lines()
    ref = oracle.run_condition(wl, ln, wl.conditions[0]).sigma
    got, st, _ = gpu_sigma(wl, ln, prec, algo=algo)
    e, l1, n = rel_err(got[0], ref)
    log(f"[pv] kind={kind} {case} prec={prec} algo={algo}: max_rel={e:.2e} L1={l1:.2e} bins={n}")
    assert n > (300 if case == "lowP" else 1000)  # 300 K Doppler widths are a fraction of a bin
    assert e <= (1e-10 if prec == FP64 else 1e-4)


def test_pseudo_voigt_adjoint_unsupported():
    import torch
    P = X()
    wl = _wl(synth.PV_OLIVERO, "mid")
    ln = wl.lines()
    plan = make_plan(wl, FP32, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    g = torch.zeros((1, wl.grid.n_bins), dtype=torch.float64, device="cuda")
    with pytest.raises(P.XsecError) as ei:
        plan.adjoint(ds, dl, g)
    assert ei.value.code == P.XS_EUNSUPPORTED
    plan.close()
