"""The allocation-free entry point xs_cross_section_noalloc (static scratch
per GPU) against xs_cross_section on the same plan and inputs: two calls in a
row, the second with fewer lines (and with accumulation), FP64 and FP32
Voigt; the FP64 results agree to 1e-12 (only the split of tiles into work
items differs), FP32 to 1e-6, on every grid point above 1e-6 of the peak and
exactly where either is zero.  A plan whose layout exceeds the scratch is
refused, and the plan's own workspace keeps the records of its last
prepare."""
import numpy as np
import pytest

import synth
from xs_helpers import X, gpu_inputs, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_noalloc_matches_cross_section(prec):
    import torch
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=12000, nu_hi=800.0, seed=2077,
                      conditions=[synth.Condition(1800.0, 0.8, 25.0), synth.Condition(2600.0, 4.0, 25.0)])
    ln = wl.lines()
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    small = ln.take(np.arange(0, ln.n, 3))
    dls = X().DeviceLines.from_numpy(small)
    tol = 1e-12 if prec == FP64 else 1e-6
    out = torch.full((2, wl.grid.n_bins), -1.0, dtype=torch.float64, device="cuda")
    for k, (lines, acc) in enumerate(((dl, False), (dls, False), (dls, True))):
        ref = plan.cross_section(ds, lines)
        if acc:
            ref = ref + ref
        torch.cuda.synchronize()
        plan.cross_section_noalloc(ds, lines, out, accumulate=acc)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        for c in range(2):
            e, l1, n = rel_err(got[c], want[c])
            log(f"[noalloc] prec={prec} call {k} cond {c}: max_rel={e:.2e} over {n} points")
            assert n > 1000 and e <= tol
            np.testing.assert_array_equal(got[c] == 0.0, want[c] == 0.0)
    # the workspace still holds the records of a prepare made before the
    # allocation-free call
    plan.prepare(ds, dl)
    plan.cross_section_noalloc(ds, dls, out)
    again = plan.profile()
    full = make_plan(wl, prec, ln.n).cross_section(ds, dl)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(again.cpu().numpy(), full.cpu().numpy())
    plan.close()


def test_noalloc_refuses_a_plan_beyond_the_scratch():
    P = X()
    wl = synth.workload("voigt_1e7", n_states=1000, n_lines=1000, nu_hi=100.0)
    ln = wl.lines()
    plan = make_plan(wl, FP32, 5_000_000)   # ~0.7 GB of workspace
    ds, dl = gpu_inputs(wl, ln)
    import torch
    out = torch.empty((1, wl.grid.n_bins), dtype=torch.float64, device="cuda")
    with pytest.raises(P.XsecError) as e:
        plan.cross_section_noalloc(ds, dl, out)
    assert e.value.code == P.XS_EWORKSPACE
    plan.close()
