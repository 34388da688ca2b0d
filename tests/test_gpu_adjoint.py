"""The hand-written adjoint (xs_cross_section_adjoint) on the GPU.

1. Against the oracle's analytic gradient for the same seeded cotangent
   dL/dsigma (both sides take the identical g): per-condition dL/dT, dL/dP
   and per-line dL/d(gamma_ref, n_exp, log_scale).  Tolerances: FP64 form
   1e-8 relative on the scalars; FP32 form 1e-3.  Per-line vectors (FP64
   1e-9, FP32 1e-4): in ||diff||_2/||ref||_2, and per element against the
   scale of each line's window sum (the same gradient with every term in
   absolute value) and in plain relative error where the sum does not
   cancel (xs_helpers.check_line_gradients); with a positive cotangent the
   log-scale gradient's sums cannot cancel, and every element with |ref| at
   least 1e-6 of the largest is held to the plain relative tolerance.
   Cotangents of 1e-30 and 1e+10 times the seeded one, and the workload's own
   cotangent 2 w (sigma - t) at its physical magnitude (~1e-20), give the
   same accuracy.
2. The adjoint workload: L = sum_k w_k (sigma_k - t_k)^2, t from T = 1700 K,
   P = 0.8 bar, w = 10^U(-2,2); dL/dT and dL/dP against central differences
   (h = 1e-3 relative) of the FP64 forward on the GPU.
3. XsecFunction (torch.autograd.Function): backward equals the adjoint.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, check_line_gradients, gpu_inputs, log, make_plan, workload

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


def _norm_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_ORACLE = {}
_WIDE = (synth.Condition(1900.0, 0.7, 25.0), synth.Condition(2500.0, 3.0, 25.0))
# low pressures, for the adjoint's block-summed forms (a level's form when
# every line of a wave of 64 neighbouring lines has y^2 at most half the
# level's rho bound).  Waves with every y^2 <= 32 / 450 (FP32 two- / one-pair
# levels): 81% / 95% at 0.05 bar, 24% / 79% at 0.2 bar, 0% / 22% at 0.7 bar;
# FP64 (<= 200 / 3200 for the three- / two-pair levels): 92% / 98%, 70% / 92%
# and 1% / 70%
_NARROW = (synth.Condition(2200.0, 0.05, 25.0), synth.Condition(2200.0, 0.2, 25.0))


def _adj_case(prof, conds=_WIDE, gscale=1.0, positive=False):
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=8000, nu_hi=600.0, profile=prof, conditions=list(conds))
    ln = wl.lines()
    rng = np.random.default_rng(31)
    ls = (0.1 * rng.standard_normal(ln.n)).astype(np.float32)
    g = wl.cotangent()
    if positive:
        g = np.abs(g)
    g = g * gscale
    key = (prof, tuple((c.T, c.P) for c in conds), gscale, positive)
    if key not in _ORACLE:
        _ORACLE[key] = [(oracle.adjoint(wl, ln, cond, g[c], log_scale=ls),
                         oracle.adjoint_bounds(wl, ln, cond, g[c], log_scale=ls))
                        for c, cond in enumerate(wl.conditions)]
    return wl, ln, ls, g, _ORACLE[key]


@pytest.mark.parametrize("prof", [synth.VOIGT, synth.DOPPLER, synth.LORENTZ])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_adjoint_vs_oracle_gradient(prof, prec):
    _check_adjoint(prof, prec, _WIDE)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_adjoint_vs_oracle_gradient_narrow_lines(prec):
    _check_adjoint(synth.VOIGT, prec, _NARROW)


@pytest.mark.parametrize("gscale", [1e-30, 1e10])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_adjoint_cotangent_magnitudes(prec, gscale):
    """The FP32 form scales each condition's cotangent by a power of two
    before its FP32 sums: tiny and huge losses keep the accuracy."""
    _check_adjoint(synth.VOIGT, prec, _WIDE, gscale=gscale)
    _check_adjoint(synth.VOIGT, prec, _NARROW, gscale=gscale)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_adjoint_per_element_positive_cotangent(prec):
    """A positive cotangent: the log-scale gradient's window sums have terms
    of one sign, so every element above 1e-6 of the largest is checked in
    plain relative error (its bound equals |ref|)."""
    _check_adjoint(synth.VOIGT, prec, _WIDE, positive=True)


def _check_adjoint(prof, prec, conds, gscale=1.0, positive=False):
    import torch
    wl, ln, ls, g, orc = _adj_case(prof, conds, gscale, positive)
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln, log_scale=ls)
    r = plan.adjoint(ds, dl, torch.as_tensor(g, device="cuda"))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in r.items()}
    ref = {"d_log_scale": 0.0, "d_gamma_ref": 0.0, "d_n_exp": 0.0}
    bnd = dict(ref)
    for c, cond in enumerate(wl.conditions):
        o, b = orc[c]
        for k in ref:
            ref[k] = ref[k] + o[k]
            bnd[k] = bnd[k] + b[k]
        stol = 1e-8 if prec == FP64 else 1e-3
        for name, gv, ov in (("dT", got["dT"][c], o["dT"]), ("dP", got["dP"][c], o["dP"])):
            if prof == synth.DOPPLER and name == "dP":
                assert gv == 0.0 and ov == 0.0
                continue
            log(f"[adj] prof={prof} prec={prec} g*{gscale:g} cond{c} {name}: gpu={gv:.10e} oracle={ov:.10e}")
            assert gv == pytest.approx(ov, rel=stol, abs=0)
    vtol = 1e-9 if prec == FP64 else 1e-4
    for k in ref:
        if prof == synth.DOPPLER and k != "d_log_scale":
            assert np.all(got[k] == 0.0)
            continue
        check_line_gradients(f"prof={prof} prec={prec} g*{gscale:g}{' |g|' if positive else ''} {k}",
                             got[k], ref[k], bnd[k], vtol)
    if positive:
        # terms of one sign: the plain per-element relative error of every
        # element at least 1e-6 of the largest
        r, gv = ref["d_log_scale"], got["d_log_scale"]
        m = np.abs(r) >= 1e-6 * np.abs(r).max()
        e = float(np.max(np.abs(gv[m] - r[m]) / np.abs(r[m])))
        log(f"[adj] positive cotangent prec={prec}: d_log_scale per-element max_rel {e:.2e} over {int(m.sum())}")
        assert m.sum() > 1000 and e <= vtol
    plan.close()


def _loss_setup(n_lines=6000, nu_hi=500.0):
    import torch
    wl = synth.workload("voigt_fit_1e7", n_states=20000, n_lines=n_lines, nu_hi=nu_hi)
    ln = wl.lines()
    ds, dl = gpu_inputs(wl, ln)
    w = torch.as_tensor(wl.bin_weights(), device="cuda")
    tplan = make_plan(wl, FP64, ln.n, conditions=[synth.Condition(1700.0, 0.8, 25.0)])
    target = tplan.cross_section(ds, dl)[0].clone()
    return wl, ln, ds, dl, w, target


def test_adjoint_scalars_by_central_differences():
    import torch
    wl, ln, ds, dl, w, target = _loss_setup()
    T0, P0 = 2000.0, 1.0
    f64 = make_plan(wl, FP64, ln.n, conditions=[synth.Condition(T0, P0, 25.0)])

    def loss(T, P):
        f64.set_conditions([synth.Condition(T, P, 25.0)])
        s = f64.cross_section(ds, dl)[0]
        return float(torch.sum(w * (s - target) ** 2).item()), s

    L0, s0 = loss(T0, P0)
    g = (2.0 * w * (s0 - target)).reshape(1, -1)
    fd_T = (loss(T0 * (1 + 1e-3), P0)[0] - loss(T0 * (1 - 1e-3), P0)[0]) / (2e-3 * T0)
    fd_P = (loss(T0, P0 * (1 + 1e-3))[0] - loss(T0, P0 * (1 - 1e-3))[0]) / (2e-3 * P0)
    f64.set_conditions([synth.Condition(T0, P0, 25.0)])
    for prec in (FP64, FP32):
        plan = make_plan(wl, prec, ln.n, conditions=[synth.Condition(T0, P0, 25.0)])
        r = plan.adjoint(ds, dl, g)
        dT, dP = float(r["dT"][0].item()), float(r["dP"][0].item())
        log(f"[fd] prec={prec} dT adj={dT:.8e} fd={fd_T:.8e}; dP adj={dP:.8e} fd={fd_P:.8e}")
        assert dT == pytest.approx(fd_T, rel=2e-4, abs=0)
        assert dP == pytest.approx(fd_P, rel=2e-4, abs=0)
        plan.close()


def test_adjoint_physical_cotangent():
    """The adjoint workload's own cotangent g = 2 w (sigma - t) at its
    physical magnitude (sigma ~ 1e-20 cm^2/molecule), with sigma and the
    target t from the oracle: per-line gradients and dL/dT, dL/dP against the
    oracle's gradient."""
    import torch
    wl = synth.workload("voigt_fit_1e7", n_states=20000, n_lines=6000, nu_hi=500.0)
    ln = wl.lines()
    cond = wl.conditions[0]
    s = oracle.run_condition(wl, ln, cond).sigma
    t = oracle.run_condition(wl, ln, synth.Condition(1700.0, 0.8, 25.0)).sigma
    g = 2.0 * wl.bin_weights() * (s - t)
    log(f"[adj phys] max |g| = {np.abs(g).max():.3e}")
    ref = oracle.adjoint(wl, ln, cond, g)
    bnd = oracle.adjoint_bounds(wl, ln, cond, g)
    ds, dl = gpu_inputs(wl, ln)
    for prec, stol, vtol in ((FP64, 1e-8, 1e-9), (FP32, 1e-3, 1e-4)):
        plan = make_plan(wl, prec, ln.n)
        r = plan.adjoint(ds, dl, torch.as_tensor(g.reshape(1, -1), device="cuda"))
        torch.cuda.synchronize()
        for name in ("dT", "dP"):
            gv = float(r[name][0].item())
            log(f"[adj phys] prec={prec} {name}: gpu={gv:.10e} oracle={ref[name]:.10e}")
            assert gv == pytest.approx(ref[name], rel=stol, abs=0)
        for k in ("d_log_scale", "d_gamma_ref", "d_n_exp"):
            check_line_gradients(f"physical cotangent prec={prec} {k}", r[k].cpu().numpy(), ref[k], bnd[k], vtol)
        plan.close()


def test_autograd_function_two_applies_one_backward():
    """Two applies of XsecFunction on one plan at different conditions before
    one backward: each backward runs the adjoint at its own forward's
    conditions."""
    import torch
    P = X()
    wl, ln, ds, dl, w, target = _loss_setup(n_lines=3000, nu_hi=300.0)
    plan = make_plan(wl, FP64, ln.n)
    gref = dl.gamma_ref.clone()
    nexp = dl.n_exp.clone()
    ls = torch.zeros(ln.n, dtype=torch.float32, device="cuda")
    TA = torch.tensor([2000.0], dtype=torch.float64, device="cuda", requires_grad=True)
    TB = torch.tensor([1500.0], dtype=torch.float64, device="cuda", requires_grad=True)
    Pr = torch.tensor([1.0], dtype=torch.float64, device="cuda")
    sA = P.XsecFunction().apply(TA, Pr, gref, nexp, ls, plan, ds, dl, [25.0])
    sB = P.XsecFunction().apply(TB, Pr, gref, nexp, ls, plan, ds, dl, [30.0])
    L = torch.sum(w * (sA[0] - target) ** 2) + torch.sum(w * sB[0] ** 2)
    L.backward()
    # each backward against the adjoint of a plan held at that forward's
    # conditions, for the same cotangent (same kernels: relative 1e-12)
    dts = []
    for T0, cut, grad, gsig in ((2000.0, 25.0, TA.grad, 2.0 * w * (sA[0].detach() - target)),
                                (1500.0, 30.0, TB.grad, 2.0 * w * sB[0].detach())):
        ref_plan = make_plan(wl, FP64, ln.n, conditions=[synth.Condition(T0, 1.0, cut)])
        r = ref_plan.adjoint(ds, P.DeviceLines(dl.upper, dl.lower, dl.einstein_a, gref, nexp, ls),
                             gsig.reshape(1, -1))
        dts.append(float(r["dT"][0].item()))
        log(f"[autograd two] T={T0} cut={cut} dL/dT autograd={grad.item():.10e} adjoint={dts[-1]:.10e}")
        assert grad.item() == pytest.approx(dts[-1], rel=1e-12, abs=0)
        ref_plan.close()
    # the first backward at the second forward's conditions would differ
    wrong = make_plan(wl, FP64, ln.n, conditions=[synth.Condition(1500.0, 1.0, 30.0)])
    rw = wrong.adjoint(ds, P.DeviceLines(dl.upper, dl.lower, dl.einstein_a, gref, nexp, ls),
                       (2.0 * w * (sA[0].detach() - target)).reshape(1, -1))
    assert abs(float(rw["dT"][0].item()) - dts[0]) > 1e-3 * abs(dts[0])
    wrong.close()
    plan.close()


def test_autograd_function_backward_is_adjoint():
    import torch
    P = X()
    wl, ln, ds, dl, w, target = _loss_setup(n_lines=3000, nu_hi=300.0)
    plan = make_plan(wl, FP32, ln.n)
    T = torch.tensor([2000.0], dtype=torch.float64, device="cuda", requires_grad=True)
    Pr = torch.tensor([1.0], dtype=torch.float64, device="cuda", requires_grad=True)
    gref = dl.gamma_ref.clone().requires_grad_(True)
    nexp = dl.n_exp.clone().requires_grad_(True)
    ls = torch.zeros(ln.n, dtype=torch.float32, device="cuda", requires_grad=True)
    sigma = P.XsecFunction().apply(T, Pr, gref, nexp, ls, plan, ds, dl, [25.0])
    L = torch.sum(w * (sigma[0] - target) ** 2)
    L.backward()
    g = (2.0 * w * (sigma[0].detach() - target)).reshape(1, -1)
    r = plan.adjoint(ds, P.DeviceLines(dl.upper, dl.lower, dl.einstein_a, gref.detach(), nexp.detach(),
                                       ls.detach()), g)
    # same kernels on both routes: relative agreement only (the gradients are ~1e-30)
    assert torch.allclose(T.grad, r["dT"], rtol=1e-12, atol=0) and torch.allclose(Pr.grad, r["dP"], rtol=1e-12, atol=0)
    assert torch.allclose(gref.grad, r["d_gamma_ref"].float(), rtol=1e-6, atol=0)
    assert torch.allclose(ls.grad, r["d_log_scale"].float(), rtol=1e-6, atol=0)
    assert T.grad.abs().item() > 0 and gref.grad.abs().max().item() > 0
    log(f"[autograd] dL/dT={T.grad.item():.6e} dL/dP={Pr.grad.item():.6e}")
    plan.close()
