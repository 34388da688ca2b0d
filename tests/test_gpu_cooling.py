"""Cooling function W(T), Eq. (cf), on the GPU against the oracle.

The GPU groups lines by upper state and sums states x temperatures; the oracle
sums lines x temperatures as printed.  Tolerance 1e-12 relative: the GPU forms
the exponent as (-c2 E) (1/T) where the oracle divides, at most two roundings
apart, i.e. 2 |x| 1.1e-16 <= 1.7e-13 relative per term for |x| <= 745, the
largest exponent with a nonzero FP64 result; every term is positive.  Cases: a
reduced benchmark line list on a temperature grid that includes 1-10 K (few
states populated); discarded and invalid lines; no lines; repeatability; the
1e7-line, 1e6-state list on the full 1-5000 K grid at sampled temperatures.
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, gpu_inputs, log, make_plan

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
TGRID = np.concatenate([[1.0, 2.0, 5.0, 10.0, 30.0, 77.0], np.arange(100.0, 5001.0, 150.0)])


def _cmp(tag, got, ref, tol=1e-12):
    m = np.abs(ref) > 1e-290
    e = float(np.max(np.abs(got[m] - ref[m]) / np.abs(ref[m]))) if m.any() else 0.0
    log(f"[cooling {tag}] max_rel={e:.2e} over {m.sum()} temperatures")
    assert e <= tol
    assert np.all(got[~m] == ref[~m]) or np.all(np.abs(got[~m]) < 1e-280)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_cooling_small(prec):
    import torch
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=200000, seed=1204)
    ln = wl.lines()
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    W, Q = plan.cooling_function(ds, dl, TGRID)
    torch.cuda.synchronize()
    Wr, Qr = oracle.cooling(wl.states, ln, TGRID)
    _cmp("small W", W.cpu().numpy(), Wr)
    _cmp("small Q", Q.cpu().numpy(), Qr)
    st = plan.stats()
    assert st["lines_kept"] == ln.n and st["lines_invalid"] == 0
    # repeatable bit for bit
    W2, _ = plan.cooling_function(ds, dl, TGRID)
    assert torch.equal(W, W2)
    # the records of a prepare are gone: a profile pass needs a new prepare
    P = X()
    with pytest.raises(P.XsecError) as ei:
        plan.profile()
    assert ei.value.code == P.XS_EINVAL
    plan.close()


def test_cooling_discarded_and_invalid_lines():
    import torch
    P = X()
    wl = synth.workload("voigt_1e7", n_states=5000, n_lines=30000, seed=1205)
    ln = wl.lines()
    n = ln.n
    up, lo = ln.upper.copy(), ln.lower.copy()
    up[:100], lo[:100] = ln.lower[:100], ln.upper[:100]     # nu < 0
    lo[100:150] = up[100:150]                                 # nu = 0
    up[150:170] = wl.states.n + 7                             # index outside the table
    bad = synth.Lines(up, lo, ln.einstein_a, ln.gamma_ref, ln.n_exp)
    plan = make_plan(wl, FP64, n)
    ds, dl = gpu_inputs(wl, bad)
    W, Q = plan.cooling_function(ds, dl, TGRID)
    torch.cuda.synchronize()
    keep = np.ones(n, bool)
    keep[150:170] = False
    Wr, Qr = oracle.cooling(wl.states, bad.take(np.nonzero(keep)[0]), TGRID)
    _cmp("discarded W", W.cpu().numpy(), Wr)
    st = plan.stats()
    assert st["lines_invalid"] == 20 and st["lines_kept"] == n - 170
    # no lines at all: W = 0, Q still the partition function
    empty = synth.Lines(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    W0, Q0 = plan.cooling_function(ds, P.DeviceLines.from_numpy(empty), TGRID[:5])
    torch.cuda.synchronize()
    assert np.all(W0.cpu().numpy() == 0.0)
    _cmp("no lines Q", Q0.cpu().numpy(), Qr[:5])
    # argument errors
    for T in ([], [300.0, -1.0], [float("nan")]):
        with pytest.raises(P.XsecError) as ei:
            plan.cooling_function(ds, dl, T)
        assert ei.value.code == P.XS_EINVAL
    plan.close()


def test_cooling_non_lte_unsupported():
    P = X()
    wl = synth.workload("twotemp_1e9", n_states=2000, n_lines=1000, n_chunks=1)
    ln = wl.lines()
    plan = make_plan(wl, FP64, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    with pytest.raises(P.XsecError) as ei:
        plan.cooling_function(ds, dl, [1000.0])
    assert ei.value.code == P.XS_EUNSUPPORTED
    plan.close()


def test_cooling_full_size():
    import torch
    wl = synth.workload("voigt_1e7")
    ln = wl.lines()
    plan = make_plan(wl, FP32, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    T = np.arange(1.0, 5001.0)
    W, Q = plan.cooling_function(ds, dl, T)
    torch.cuda.synchronize()
    W, Q = W.cpu().numpy(), Q.cpu().numpy()
    idx = np.array([0, 9, 99, 295, 999, 1999, 3499, 4999])
    Wr, Qr = oracle.cooling(wl.states, ln, T[idx])
    _cmp("full W", W[idx], Wr)
    _cmp("full Q", Q[idx], Qr)
    assert np.all(np.diff(W[100:]) > 0)  # more hot emitters as T rises
    plan.close()
