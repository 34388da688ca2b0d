"""Parity of the 48-condition opacity grid at its full size, in the launch
form the benchmark times for it: 1e8 lines and 1e6 states, LTE Voigt
absorption at T in {300 ... 5000 K} x P in {1e-4 ... 100 bar} (cut-off 25
cm^-1, or 100 cm^-1 at P >= 10 bar), grid 0-20000 cm^-1 step 0.01, all 48
conditions in one captured graph (intensities, bucketing, one persistent
profile launch), FP32 and FP64 forms.

The oracle cannot afford 48 full grids over 1e8 lines, so it computes sigma
at sampled grid points of each condition, all chosen on the oracle's side
(never from the GPU's output):
* in four random sub-bands of 200 cm^-1 shared by every condition, the home
  point and the points 1 and 3 steps either side of the six strongest lines
  of each sub-band by the oracle's own intensities at the condition's
  temperature (the intensities do not depend on P);
* six uniform random points in each sub-band.
The comparison threshold is 1e-6 of the largest oracle value over those
points; every condition must compare at least 50 of them.  For each
condition the oracle receives only the lines whose window can reach one of
the points (a superset, taken from coarse 1 cm^-1 buckets of the
wavenumbers), which leaves its sums unchanged.
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import gpu_inputs, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
BANDS, BAND_CM, STRONG, UNIFORM = 4, 200, 6, 6
OFFSETS = np.array([-3, -1, 0, 1, 3])


@pytest.fixture(scope="module")
def grid48():
    import torch
    wl = synth.workload("voigt_grid48_1e8")
    ln = wl.lines()
    log(f"[full48] {ln.n} lines, {len(wl.conditions)} conditions generated")
    ds, dl = gpu_inputs(wl, ln)
    out = {}
    for prec, name in ((FP32, "f32"), (FP64, "f64")):
        p = make_plan(wl, prec, ln.n)
        sig = torch.empty((len(wl.conditions), wl.grid.n_bins), dtype=torch.float64, device="cuda")
        p.capture(ds, dl, sig)
        p.replay()
        torch.cuda.synchronize()
        out[name] = sig.cpu().numpy()
        log(f"[full48] {name} graph replayed")
        p.close()
        del sig
    del ds, dl
    torch.cuda.empty_cache()
    # coarse buckets of the wavenumbers, to hand the oracle only nearby lines
    E = wl.states.energy
    nu = E[ln.upper] - E[ln.lower]
    key = np.clip(np.floor(nu), -1, 20001).astype(np.int16)
    order = np.argsort(key, kind="stable")
    start = np.searchsorted(key[order], np.arange(-1, 20003), side="left")
    del nu
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(4803)))
    bands = rng.integers(100, 20000 - BAND_CM - 100, BANDS)
    # the strongest lines of each sub-band by the oracle's intensities, per
    # distinct temperature
    strong = {}
    for T in sorted({c.T for c in wl.conditions}):
        Q, _ = oracle.partition(wl.states, wl.population, T)
        ks = []
        for b in bands:
            idx = order[start[b + 1]:start[b + 1 + BAND_CM]]
            nu_b, S_b, _ = oracle.intensities(wl.states, ln.take(idx), wl.mode, wl.population, T, Q)
            top = np.argpartition(S_b, -STRONG)[-STRONG:]
            ks.append(np.rint((nu_b[top] - wl.grid.nu0) / wl.grid.dnu).astype(np.int64))
        strong[T] = np.concatenate(ks)
    return wl, ln, out, order, start, bands, strong


def _nearby_lines(wl, order, start, bins, cut):
    """Indices of every line whose wavenumber lies within cut + 2 cm^-1 of a
    point in bins (bucket b holds wavenumbers in [b, b + 1))."""
    want = np.zeros(20003, bool)
    for k in bins:
        nu_k = wl.grid.nu0 + k * wl.grid.dnu
        lo = max(int(np.floor(nu_k - cut)) - 2, -1)
        hi = min(int(np.floor(nu_k + cut)) + 2, 20001)
        want[lo + 1:hi + 2] = True
    runs = np.flatnonzero(np.diff(np.concatenate([[0], want.astype(np.int8), [0]])))
    parts = [order[start[a]:start[b]] for a, b in zip(runs[::2], runs[1::2])]
    return np.sort(np.concatenate(parts))


def _points(wl, bands, strong, ci):
    """Sampled points of condition ci (see the module docstring)."""
    cond = wl.conditions[ci]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([4803, ci])))
    pts = [(strong[cond.T][:, None] + OFFSETS[None, :]).ravel()]
    per = int(round(BAND_CM / wl.grid.dnu))
    for b in bands:
        k0 = int(round((b - wl.grid.nu0) / wl.grid.dnu))
        pts.append(k0 + rng.integers(0, per, UNIFORM))
    bins = np.unique(np.concatenate(pts))
    return bins[(bins >= 0) & (bins < wl.grid.n_bins)]


def _check(grid48, conds):
    wl, ln, out, order, start, bands, strong = grid48
    n_total = 0
    for ci in conds:
        cond = wl.conditions[ci]
        s64, s32 = out["f64"][ci], out["f32"][ci]
        bins = _points(wl, bands, strong, ci)
        idx = _nearby_lines(wl, order, start, bins, cond.cutoff)
        ref = oracle.run_condition(wl, ln.take(idx), cond, bins=bins).sigma
        peak = float(ref.max())
        for name, got, tol in (("fp64", s64, 1e-10), ("fp32", s32, 1e-4)):
            e, l1, n = rel_err(got[bins], ref, peak=peak)
            log(f"[full48] T={cond.T:g} P={cond.P:g} {name}: max_rel={e:.2e} over {n} of "
                f"{len(bins)} points ({len(idx)} lines)")
            assert n >= 50, (ci, name, n)
            assert e <= tol, (ci, name, e)
        n_total += n
    return n_total


@pytest.mark.parametrize("part", range(4))
def test_batched_grid_full_size(grid48, part):
    """Conditions 12 part ... 12 part + 11 (T ascending, P ascending within T)."""
    n = _check(grid48, range(12 * part, 12 * part + 12))
    assert n >= 600
