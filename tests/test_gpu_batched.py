"""The batched opacity grid: all 48 (T, P) conditions of the batched workload
(T in 8 values x P in 6 values, cut-off 100 cm^-1 at P >= 10 bar) in one plan,
run through a captured graph (intensities, bucketing and one persistent
profile launch for every condition), on the full 2,000,001-point grid with a
reduced line list; every condition is compared with the oracle at sampled
grid points, its peak and the points around its strongest lines, in the
FP32 and FP64 forms."""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import gpu_inputs, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_batched_48_conditions_graph_vs_oracle(prec):
    import torch
    wl = synth.workload("voigt_grid48_1e8", n_lines=200_000, n_states=100_000)
    assert len(wl.conditions) == 48
    ln = wl.lines()
    ds, dl = gpu_inputs(wl, ln)
    plan = make_plan(wl, prec, ln.n)
    sig = torch.zeros((48, wl.grid.n_bins), dtype=torch.float64, device="cuda")
    plan.capture(ds, dl, sig)
    sig.fill_(-1.0)
    plan.replay()
    torch.cuda.synchronize()
    bins = synth.sample_bins(wl.grid.n_bins, 4000, 11)
    tb = torch.as_tensor(bins, device="cuda")
    peaks = torch.argmax(sig, dim=1).cpu().numpy()
    got_all = sig[:, tb].cpu().numpy()
    worst = 0.0
    for c, cond in enumerate(wl.conditions):
        # random points, the peak, and the points around the 200 strongest
        # lines (from the oracle's own intensities): at low T and P the
        # profiles are so narrow that random points mostly fall in far wings
        r0 = oracle.run_condition(wl, ln, cond, with_sigma=False)
        top = np.argsort(r0.S)[-200:]
        kc = np.rint((r0.nu[top] - wl.grid.nu0) / wl.grid.dnu).astype(np.int64)
        near = (kc[:, None] + np.array([-3, -1, 0, 1, 3])[None, :]).ravel()
        near = near[(near >= 0) & (near < wl.grid.n_bins)]
        b = np.unique(np.concatenate([bins, [peaks[c]], near]))
        got = sig[c, torch.as_tensor(b, device="cuda")].cpu().numpy()
        ref = oracle.run_condition(wl, ln, cond, bins=b).sigma
        e, l1, n = rel_err(got, ref)
        worst = max(worst, e)
        assert n > 200, (cond, n)
        assert e <= (1e-10 if prec == FP64 else 1e-4), (cond, e)
        if c % 8 == 0:
            log(f"[batched] prec={prec} T={cond.T} P={cond.P} cut={cond.cutoff}: max_rel={e:.2e} L1={l1:.2e} n={n}")
    assert np.all(got_all >= 0.0)
    log(f"[batched] prec={prec} 48 conditions, worst max_rel {worst:.2e}")
    plan.close()
