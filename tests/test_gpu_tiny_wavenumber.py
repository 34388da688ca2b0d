"""Lines with tiny wavenumbers (nu = E_u - E_l from 1e-7 to 1e-2 cm^-1) mixed
into an ordinary Voigt list, on the GPU against the oracle.

Their Doppler width scales with nu, so for them x = (nu_k - nu)/(sg sqrt 2)
reaches 1e9 and more across a 25 cm^-1 window and y = gamma/(sg sqrt 2)
reaches 1e11: the FP32 gather and adjoint evaluate such lines in FP64, the
FP64 gather sends them to its per-chunk path (its far rows share one
reciprocal among four points only while |x|, y <= 1e9), and the FP64
adjoint keeps one reciprocal per point in the waves that hold them.  Their
Einstein A is scaled by nu so that their intensities (which grow as 1/nu)
stay comparable with the other lines'.

Tolerances as in test_gpu_parity (sigma: 1e-10 FP64, 1e-4 FP32 over points
at or above 1e-6 of the peak) and test_gpu_adjoint (dT, dP: 1e-8 / 1e-3;
per-line vectors 1e-9 / 1e-4, norm and per element).
"""
import copy

import numpy as np
import pytest

import oracle
import synth
from xs_helpers import check_line_gradients, gpu_inputs, gpu_sigma, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
_CASE = {}


def _case():
    """3000 ordinary lines on 0-100 cm^-1 plus 120 lines whose upper state
    lies 1e-7 ... 1e-2 cm^-1 above its lower state (new states appended)."""
    if not _CASE:
        wl = synth.workload("voigt_1e7", n_states=5000, n_lines=3000, nu_hi=100.0, seed=91)
        ln = wl.lines()
        rng = np.random.default_rng(5)
        n = 120
        delta = np.array([1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7])[rng.integers(0, 6, n)]
        lower = rng.integers(1, wl.states.n, n)
        E = np.concatenate([wl.states.energy, wl.states.energy[lower] + delta])
        g = np.concatenate([wl.states.g_tot, wl.states.g_tot[lower]])
        upper = np.arange(wl.states.n, wl.states.n + n, dtype=np.int32)
        lines = synth.Lines(np.concatenate([ln.upper, upper]).astype(np.int32),
                            np.concatenate([ln.lower, lower.astype(np.int32)]),
                            np.concatenate([ln.einstein_a, (ln.einstein_a[:n] * delta).astype(np.float32)]),
                            np.concatenate([ln.gamma_ref, ln.gamma_ref[:n]]),
                            np.concatenate([ln.n_exp, ln.n_exp[:n]]))
        w2 = copy.copy(wl)
        w2.states = synth.States(E, g)
        w2._lines_cache = lines
        _CASE["wl"], _CASE["lines"] = w2, lines
        _CASE["sigma"] = oracle.run_condition(w2, lines, w2.conditions[0]).sigma
        gc = w2.cotangent()
        _CASE["g"] = gc
        _CASE["adj"] = oracle.adjoint(w2, lines, w2.conditions[0], gc[0])
        _CASE["bound"] = oracle.adjoint_bounds(w2, lines, w2.conditions[0], gc[0])
    return _CASE


@pytest.mark.parametrize("algo", [0, 1])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_sigma_tiny_wavenumbers(prec, algo):
    c = _case()
    got, st, _ = gpu_sigma(c["wl"], c["lines"], prec, algo=algo)
    ref = c["sigma"]
    e, l1, n = rel_err(got[0], ref)
    log(f"[tiny nu] algo={algo} prec={'fp32' if prec else 'fp64'} max_rel={e:.3e} L1={l1:.3e} bins={n} "
        f"(peak at point {int(np.argmax(ref))})")
    assert n > 1000
    assert e <= (1e-10 if prec == FP64 else 1e-4)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_adjoint_tiny_wavenumbers(prec):
    import torch
    c = _case()
    wl, lines = c["wl"], c["lines"]
    plan = make_plan(wl, prec, lines.n)
    ds, dl = gpu_inputs(wl, lines)
    r = plan.adjoint(ds, dl, torch.as_tensor(c["g"], device="cuda"))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in r.items()}
    plan.close()
    o, b = c["adj"], c["bound"]
    stol = 1e-8 if prec == FP64 else 1e-3
    for name in ("dT", "dP"):
        log(f"[tiny nu adj] prec={prec} {name}: gpu={got[name][0]:.10e} oracle={o[name]:.10e}")
        assert got[name][0] == pytest.approx(o[name], rel=stol, abs=0)
    vtol = 1e-9 if prec == FP64 else 1e-4
    for k in ("d_log_scale", "d_gamma_ref", "d_n_exp"):
        check_line_gradients(f"tiny nu prec={prec} {k}", got[k], o[k], b[k], vtol)
