"""Properties of the GPU pipeline through the C-ABI: the captured graph
replays the eager result; the FP64 gather is bitwise repeatable (and both
forms on narrow Doppler lines, which take the LDS row path); every kernel
configuration the autotuner may pick gives the same sigma (within the
tolerance of the form); chunked accumulation equals the whole line list;
batched conditions equal separate runs; edge cases (no lines, all lines
discarded, one grid point, lines beyond the grid, invalid state indices)."""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, gpu_inputs, log, make_plan, rel_err, workload

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


def _voigt_small():
    return workload("voigt_1e7", n_states=20000, n_lines=20000, nu_hi=1200.0)


def test_graph_replay_equals_eager():
    import torch
    wl = _voigt_small()
    ln = wl.lines()
    for prec in (FP64, FP32):
        plan = make_plan(wl, prec, ln.n)
        ds, dl = gpu_inputs(wl, ln)
        eager = plan.cross_section(ds, dl).clone()
        out = torch.full_like(eager, -1.0)
        plan.capture(ds, dl, out)
        for rep in range(3):
            out.fill_(-1.0)
            plan.replay()
            torch.cuda.synchronize()
            tmp = torch.empty_like(eager).fill_(3.0)  # eager work between replays
            assert torch.equal(out, eager), f"replay {rep} differs"
        log(f"[graph] prec={prec} 3 replays bitwise equal to eager")
        plan.close()


def test_gather_fp64_bitwise_repeatable_and_scatter_close():
    import torch
    wl = _voigt_small()
    ln = wl.lines()
    plan = make_plan(wl, FP64, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    a = plan.cross_section(ds, dl).clone()
    b = plan.cross_section(ds, dl).clone()
    assert torch.equal(a, b)
    ps = make_plan(wl, FP64, ln.n, algo=1)
    s = ps.cross_section(ds, dl)
    e, _, _ = rel_err(s[0].cpu().numpy(), a[0].cpu().numpy())
    log(f"[repeat] fp64 gather bitwise repeatable; scatter vs gather {e:.2e}")
    # The gather's far rows (|z|^2 >= 4000, so |x| >= 63) step x from the
    # row's first point, the scatter forms (nu_k - nu) inv at every point:
    # they differ by the rounding of nu_k, at most ~1e-10 absolute in x here,
    # which moves a value by at most 2 |dx| / |x| <= 3.2e-12 relative; the
    # node rules of the two paths agree within 2e-13.  Every term is positive,
    # so the sums differ by at most as much.
    assert e < 4e-12


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_gaussian_rows_repeatable_and_replayed(prec):
    """Narrow Doppler lines go through the per-lane LDS row adds: two eager
    runs are bitwise equal, and so are three graph replays."""
    import torch
    wl = workload("twotemp_1e9", n_states=20000, n_lines=30000, n_chunks=1, nu_hi=2000.0)
    ln = wl.lines()
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    a = plan.cross_section(ds, dl).clone()
    b = plan.cross_section(ds, dl).clone()
    assert torch.equal(a, b)
    out = torch.full_like(a, -1.0)
    plan.capture(ds, dl, out)
    for rep in range(3):
        out.fill_(-1.0)
        plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, a), f"replay {rep} differs"
    log(f"[gauss rows] prec={prec}: eager runs and 3 replays bitwise equal")
    plan.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_all_configurations_agree(prec):
    import torch
    wl = _voigt_small()
    ln = wl.lines()
    ref = oracle.run_condition(wl, ln, wl.conditions[0]).sigma
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    for tile in (256, 512, 1024):
        for bucket, chunk in ((128, 0), (256, 64), (1024, 640), (256, 0), (4096, 0)):
            for pers in (0, 1):
                plan.set_config(tile_bins=tile, bucket_bins=bucket, persistent=pers, waves_per_cu=8,
                                chunk_lines=chunk)
                got = plan.cross_section(ds, dl)[0].cpu().numpy()
                e, _, _ = rel_err(got, ref)
                assert e <= (1e-10 if prec == FP64 else 1e-4), (tile, bucket, chunk, pers, e)
    cfg = plan.autotune(ds, dl, torch.empty((1, wl.grid.n_bins), dtype=torch.float64, device="cuda"))
    got = plan.cross_section(ds, dl)[0].cpu().numpy()
    e, _, _ = rel_err(got, ref)
    log(f"[configs] prec={prec} autotuned {cfg} err {e:.2e}")
    assert e <= (1e-10 if prec == FP64 else 1e-4)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_autotuned_doppler_plan(prec):
    """The autotuner also tries a second bucket size (here 256 points after the
    Doppler plan's 64), re-bucketing the lines in place; the tuned plan still
    matches the oracle."""
    import torch
    wl = workload("twotemp_1e9", n_states=20000, n_lines=30000, n_chunks=1, nu_hi=2000.0)
    ln = wl.lines()
    plan = make_plan(wl, prec, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    assert plan.get_config()["bucket_bins"] == 64
    cfg = plan.autotune(ds, dl, torch.empty((len(wl.conditions), wl.grid.n_bins), dtype=torch.float64,
                                            device="cuda"))
    got = plan.cross_section(ds, dl).cpu().numpy()
    for c, cond in enumerate(wl.conditions):
        ref = oracle.run_condition(wl, ln, cond).sigma
        e, _, _ = rel_err(got[c], ref)
        assert e <= (1e-10 if prec == FP64 else 1e-4), (c, cfg, e)
    log(f"[autotune doppler] prec={prec} {cfg}")
    plan.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_chunked_accumulation_equals_whole(prec):
    import torch
    wl = workload("twotemp_1e9", n_states=20000, n_lines=40000, n_chunks=4, nu_hi=2000.0)
    whole = wl.lines()
    plan = make_plan(wl, prec, max(wl.chunk_sizes()))
    ds = X().DeviceStates.from_numpy(wl.states)
    sig = torch.zeros((len(wl.conditions), wl.grid.n_bins), dtype=torch.float64, device="cuda")
    for j in range(wl.n_chunks):
        dl = X().DeviceLines.from_numpy(wl.chunk(j))
        plan.cross_section(ds, dl, out=sig, accumulate=(j > 0))
    torch.cuda.synchronize()
    got = sig.cpu().numpy()
    for c, cond in enumerate(wl.conditions):
        ref = oracle.run_condition(wl, whole, cond).sigma
        e, l1, n = rel_err(got[c], ref)
        log(f"[chunks] prec={prec} cond{c} (Tv={cond.T_vib},Tr={cond.T_rot}) max_rel={e:.2e} L1={l1:.2e}")
        assert e <= (1e-10 if prec == FP64 else 1e-4)


def test_batched_conditions_equal_separate_and_oracle():
    # Many (T, P) in one launch (the 48-point opacity grid at reduced size):
    # compare every condition on sampled bins with the oracle.
    import torch
    conds = [synth.Condition(T, P, 100.0 if P >= 10 else 25.0) for T in (300.0, 1200.0, 5000.0)
             for P in (1e-4, 1.0, 50.0)]
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=30000, nu_hi=2000.0, conditions=conds)
    ln = wl.lines()
    plan = make_plan(wl, FP32, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    sig = plan.cross_section(ds, dl)
    torch.cuda.synchronize()
    got = sig.cpu().numpy()
    bins = synth.sample_bins(wl.grid.n_bins, 400, 5)
    for c, cond in enumerate(conds):
        b = np.unique(np.concatenate([bins, [int(np.argmax(got[c]))]]))
        ref = oracle.run_condition(wl, ln, cond, bins=b).sigma
        e, _, n = rel_err(got[c][b], ref)
        log(f"[batch] T={cond.T} P={cond.P} cut={cond.cutoff} max_rel={e:.2e} bins={n}")
        assert e <= 1e-4
    # and one condition on its own plan equals its row of the batch
    single = make_plan(wl, FP32, ln.n, conditions=[conds[4]])
    s1 = single.cross_section(ds, dl)[0].cpu().numpy()
    e, _, _ = rel_err(s1, got[4])
    assert e <= 1e-6


def test_edge_cases():
    import torch
    P = X()
    wl = synth.workload("voigt_1e7", n_states=2000, n_lines=500, nu_hi=100.0)
    ln = wl.lines()
    ds, dl = gpu_inputs(wl, ln)
    # no lines
    plan = make_plan(wl, FP32, 1000)
    empty = P.DeviceLines(dl.upper[:0], dl.lower[:0], dl.einstein_a[:0], dl.gamma_ref[:0], dl.n_exp[:0])
    s = plan.cross_section(ds, empty)
    torch.cuda.synchronize()
    assert torch.count_nonzero(s).item() == 0
    # every line discarded (upper and lower swapped: nu < 0)
    sw = P.DeviceLines(dl.lower, dl.upper, dl.einstein_a, dl.gamma_ref, dl.n_exp)
    s = plan.cross_section(ds, sw)
    torch.cuda.synchronize()
    assert torch.count_nonzero(s).item() == 0 and plan.stats()["lines_kept"] == 0
    # invalid state indices are dropped and counted, not read
    bad_up = dl.upper.clone()
    bad_up[:7] = 10 ** 9
    bad_up[7:9] = -3
    bl = P.DeviceLines(bad_up, dl.lower, dl.einstein_a, dl.gamma_ref, dl.n_exp)
    plan.cross_section(ds, bl)
    torch.cuda.synchronize()
    assert plan.stats()["lines_invalid"] == 9
    plan.close()
    # a one-point grid and a grid whose lines all lie beyond its ends
    for grid in (synth.Grid(50.0, 0.01, 1), synth.Grid(150.0, 0.01, 1000), synth.Grid(-30.0, 0.01, 2001)):
        wl2 = synth.workload("voigt_1e7", n_states=2000, n_lines=500, nu_hi=100.0)
        wl2.grid = grid
        for prec in (FP64, FP32):
            plan = make_plan(wl2, prec, ln.n)
            got = plan.cross_section(ds, dl)[0].cpu().numpy()
            ref = oracle.run_condition(wl2, ln, wl2.conditions[0]).sigma
            e, _, n = rel_err(got, ref) if ref.max() > 0 else (float(np.abs(got).max()), 0, 0)
            log(f"[edge] grid nu0={grid.nu0} n={grid.n_bins} prec={prec} err={e:.2e} bins={n}")
            assert e <= (1e-10 if prec == FP64 else 1e-4)
            plan.close()


def test_host_validation_errors():
    P = X()
    wl = _voigt_small()
    ln = wl.lines()
    ds, dl = gpu_inputs(wl, ln)
    plan = make_plan(wl, FP32, 100)
    with pytest.raises(P.XsecError) as ei:
        plan.cross_section(ds, dl)  # more lines than max_lines
    assert ei.value.code == P.XS_EINVAL
    plan.close()
