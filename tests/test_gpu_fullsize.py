"""Parity at the full size of the benchmark workload, in the launch
configuration bench.py times (the autotuner's choice, read from the same
cache): 1e7 lines, 1e6 states, LTE Voigt absorption at T = 2000 K, P = 1 bar,
grid 0-20000 cm^-1 step 0.01 (2,000,001 points), cut-off 25 cm^-1.

* sigma (FP32 and FP64 forms) at sampled grid points, which the oracle
  computes one by one over all 1e7 lines: uniform draws and the points
  around the strongest lines by the oracle's intensities;
* per-line adjoint gradients (d/dlog_scale, d/dgamma_ref, d/dn_exp) of
  sampled lines against the oracle's, for the same cotangent: in norm and
  per element (xs_helpers.check_line_gradients);
* dL/dT and dL/dP of the FP32 and FP64 adjoints against central differences
  of the FP64 forward on the GPU (a property that holds at any size).
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, check_line_gradients, gpu_inputs, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
CACHE = os.path.join("/tmp", "xsec_autotune.json")


@pytest.fixture(scope="module")
def full():
    import torch
    wl = synth.workload("voigt_1e7")
    ln = wl.lines()
    ds, dl = gpu_inputs(wl, ln)
    sig = torch.empty((1, wl.grid.n_bins), dtype=torch.float64, device="cuda")
    p32 = make_plan(wl, FP32, ln.n)
    cfg = p32.autotune(ds, dl, sig, cache_path=CACHE)
    log(f"[full] config {cfg}")
    yield wl, ln, ds, dl, cfg, p32
    p32.close()


def test_sigma_sampled_points_full_size(full):
    wl, ln, ds, dl, cfg, p32 = full
    s32 = p32.cross_section(ds, dl)[0].cpu().numpy()
    p64 = make_plan(wl, FP64, ln.n)
    p64.set_config(**cfg)
    s64 = p64.cross_section(ds, dl)[0].cpu().numpy()
    p64.close()
    # sigma spans many decades, so only ~15% of uniformly drawn points are
    # above 1e-6 of the peak: draw enough of them, and add the points around
    # the 100 strongest lines by the oracle's own intensities
    cond = wl.conditions[0]
    bins = synth.sample_bins(wl.grid.n_bins, 20000, 77)
    r0 = oracle.run_condition(wl, ln, cond, with_sigma=False)
    top = np.argpartition(r0.S, -100)[-100:]
    kc = np.rint((r0.nu[top] - wl.grid.nu0) / wl.grid.dnu).astype(np.int64)
    near = (kc[:, None] + np.array([-3, -1, 0, 1, 3])[None, :]).ravel()
    bins = np.unique(np.concatenate([bins, near[(near >= 0) & (near < wl.grid.n_bins)]]))
    ref = oracle.run_condition(wl, ln, cond, bins=bins).sigma
    peak = float(ref.max())
    for name, got, tol in (("fp64", s64, 1e-10), ("fp32", s32, 1e-4)):
        e, l1, n = rel_err(got[bins], ref, peak=peak)
        log(f"[full] sigma {name}: max_rel={e:.2e} L1={l1:.2e} over {n} sampled points (peak {peak:.3e})")
        assert n > 2000
        assert e <= tol


def test_adjoint_sampled_lines_full_size(full):
    import torch
    wl, ln, ds, dl, cfg, p32 = full
    g = wl.cotangent()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(ln.n, 400, replace=False))
    sub = ln.take(idx)
    ref = oracle.adjoint(wl, sub, wl.conditions[0], g[0])
    bnd = oracle.adjoint_bounds(wl, sub, wl.conditions[0], g[0])
    p64 = make_plan(wl, FP64, ln.n)
    p64.set_config(**cfg)
    for name, plan, tol in (("fp64", p64, 1e-9), ("fp32", p32, 1e-4)):
        r = plan.adjoint(ds, dl, torch.as_tensor(g, device="cuda"))
        torch.cuda.synchronize()
        for k in ("d_log_scale", "d_gamma_ref", "d_n_exp"):
            got = r[k].cpu().numpy()[idx]
            check_line_gradients(f"full size {name} {k} ({len(idx)} sampled lines)", got, ref[k], bnd[k], tol)
    p64.close()


def test_adjoint_scalars_by_gpu_finite_differences_full_size(full):
    import torch
    wl, ln, ds, dl, cfg, p32 = full
    cond = wl.conditions[0]
    w = torch.as_tensor(wl.bin_weights(), device="cuda")

    def sigma64(T, P):
        p = make_plan(wl, FP64, ln.n, conditions=[synth.Condition(T, P, cond.cutoff)])
        p.set_config(**cfg)
        s = p.cross_section(ds, dl)[0].clone()
        p.close()
        return s

    target = sigma64(1700.0, 0.8)

    def loss(T, P):
        d = sigma64(T, P) - target
        return math.fsum((w * d * d).cpu().numpy())

    s0 = sigma64(cond.T, cond.P)
    g = (2.0 * w * (s0 - target)).reshape(1, -1)
    hT, hP = 1e-4 * cond.T, 1e-4 * cond.P
    fd_T = (loss(cond.T + hT, cond.P) - loss(cond.T - hT, cond.P)) / (2 * hT)
    fd_P = (loss(cond.T, cond.P + hP) - loss(cond.T, cond.P - hP)) / (2 * hP)
    p64 = make_plan(wl, FP64, ln.n)
    p64.set_config(**cfg)
    for name, plan, tol in (("fp64", p64, 1e-6), ("fp32", p32, 1e-4)):
        r = plan.adjoint(ds, dl, g)
        dT, dP = float(r["dT"][0].item()), float(r["dP"][0].item())
        log(f"[full] {name} dT adj={dT:.8e} fd={fd_T:.8e}  dP adj={dP:.8e} fd={fd_P:.8e}")
        assert dT == pytest.approx(fd_T, rel=tol, abs=0)
        assert dP == pytest.approx(fd_P, rel=tol, abs=0)
    p64.close()
