"""Predissociation (lifetime) broadening on the GPU against the oracle.

A third of the states of a reduced benchmark list get lifetimes
10^U(-13,-10) s (widths 0.003-2.7 cm^-1 HWHM, from well below to far above
the pressure widths), the rest are stable.  sigma (sampled and binned Voigt,
Lorentzian; gather and scatter; FP64 1e-10 and FP32 1e-4 on bins >= 1e-6 of
the peak) and the adjoint (per-line gradients and dL/dT, dL/dP against the
oracle's analytic gradient: FP64 1e-9 / 1e-8, FP32 1e-4 / 1e-3, per-line
vectors in norm and per element) with the
lifetime width entering the profile and the chain rule acting on the
pressure width only.
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import check_line_gradients, gpu_inputs, gpu_sigma, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


def _wl(profile, n_lines=3000, nu_hi=300.0, conditions=None):
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=n_lines, nu_hi=nu_hi, profile=profile, seed=1231,
                      conditions=conditions)
    return synth.with_lifetimes(wl, frac=0.33, seed=5)


@pytest.mark.parametrize("profile", [synth.VOIGT, synth.LORENTZ, synth.BIN_VOIGT])
@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("algo", [0, 1])
def test_lifetime_sigma(profile, prec, algo):
    wl = _wl(profile, n_lines=2000 if profile == synth.BIN_VOIGT else 3000)
    ln = wl.lines()
    ref = oracle.run_condition(wl, ln, wl.conditions[0]).sigma
    got, st, _ = gpu_sigma(wl, ln, prec, algo=algo)
    e, l1, n = rel_err(got[0], ref)
    log(f"[lifetime] prof={profile} prec={prec} algo={algo}: max_rel={e:.2e} L1={l1:.2e} bins={n}")
    assert n > 1000
    assert e <= (1e-10 if prec == FP64 else 1e-4)
    # the lifetimes matter: without them sigma differs well beyond the tolerance
    wl.states.lifetime = None
    plain = oracle.run_condition(wl, ln, wl.conditions[0]).sigma
    assert rel_err(plain, ref)[0] > 1e-2


@pytest.mark.parametrize("prof", [synth.VOIGT, synth.LORENTZ])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_lifetime_adjoint(prof, prec):
    import torch
    wl = _wl(prof, n_lines=6000, nu_hi=500.0,
             conditions=[synth.Condition(1900.0, 0.7, 25.0), synth.Condition(2500.0, 3.0, 25.0)])
    ln = wl.lines()
    g = wl.cotangent()
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    r = plan.adjoint(ds, dl, torch.as_tensor(g, device="cuda"))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in r.items()}
    ref = {"d_log_scale": 0.0, "d_gamma_ref": 0.0, "d_n_exp": 0.0}
    bnd = dict(ref)
    for c, cond in enumerate(wl.conditions):
        o = oracle.adjoint(wl, ln, cond, g[c])
        b = oracle.adjoint_bounds(wl, ln, cond, g[c])
        for k in ref:
            ref[k] = ref[k] + o[k]
            bnd[k] = bnd[k] + b[k]
        for name in ("dT", "dP"):
            gv, ov = float(got[name][c]), o[name]
            log(f"[lifetime adj] prof={prof} prec={prec} c{c} {name}: gpu={gv:.10e} oracle={ov:.10e}")
            assert gv == pytest.approx(ov, rel=1e-8 if prec == FP64 else 1e-3, abs=0)
    for k in ref:
        check_line_gradients(f"lifetime prof={prof} prec={prec} {k}", got[k], ref[k], bnd[k],
                             1e-9 if prec == FP64 else 1e-4)
    plan.close()
