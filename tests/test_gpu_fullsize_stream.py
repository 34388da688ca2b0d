"""Parity of the two-temperature emission workload at its full size, in the
streamed form the benchmark times for it: 1e9 lines in 10 chunks of 1e8,
generated into host memory and uploaded on a copy stream while the previous
chunk runs; 1e6 states, 4 (T_vib, T_rot) pairs, Doppler profile at T_rot,
grid 0-30000 cm^-1 step 0.05 (600,001 points), cut-off 25 cm^-1; FP32 and
FP64 forms.

The oracle computes sigma at sampled points of each condition, all chosen on
the oracle's side (never from the GPU's output): in four random sub-bands of
100 cm^-1 shared by every condition, the home point and the points 1 and 2
steps either side of the eight strongest lines of each sub-band by the
oracle's own intensities at that condition, and six uniform random points per
sub-band.  The comparison threshold is 1e-6 of the largest oracle value over
those points; every condition must compare at least 50 of them.  The oracle
receives only the lines within cut-off + 2 cm^-1 of a sampled point (taken
from 1 cm^-1 buckets of each chunk's wavenumbers), which leaves its sums
unchanged.
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
BANDS, BAND_CM, STRONG, UNIFORM = 4, 100, 8, 6
OFFSETS = np.array([-2, -1, 0, 1, 2])


@pytest.fixture(scope="module")
def stream1e9():
    import torch
    from concurrent.futures import ThreadPoolExecutor
    P = X()
    wl = synth.workload("twotemp_1e9")
    sizes = wl.chunk_sizes()
    with ThreadPoolExecutor(max_workers=min(wl.n_chunks, 16)) as ex:
        chunks = list(ex.map(wl.chunk, range(wl.n_chunks)))
    log(f"[stream1e9] {wl.n_chunks} chunks generated")
    ds = P.DeviceStates.from_numpy(wl.states)
    out = {}
    for prec, name in ((FP32, "f32"), (FP64, "f64")):
        plan = make_plan(wl, prec, max(sizes))
        sig = torch.zeros((len(wl.conditions), wl.grid.n_bins), dtype=torch.float64, device="cuda")
        st = P.ChunkStreamer(plan, max(sizes))
        n = st.run(ds, chunks, sig)
        torch.cuda.synchronize()
        assert n == sum(sizes)
        out[name] = sig.cpu().numpy()
        log(f"[stream1e9] {name}: {n} lines streamed")
        st.close()
        del st, sig
        plan.close()
    torch.cuda.empty_cache()
    return wl, chunks, out


def _strong_and_points(wl, chunks, bands):
    """Per condition: the sampled points (module docstring), from the
    oracle's intensities of the lines in the sub-bands, chunk by chunk."""
    E = wl.states.energy
    nb = int(np.ceil(wl.grid.nu0 + wl.grid.n_bins * wl.grid.dnu)) + 3
    inband = np.zeros(nb + 1, bool)
    for b in bands:
        inband[b + 1:b + 1 + BAND_CM] = True
    cand = [[] for _ in wl.conditions]  # per condition: (nu, S) of the best lines so far
    for ch in chunks:
        nu = E[ch.upper] - E[ch.lower]
        key = np.clip(np.floor(nu), -1, nb - 1).astype(np.int32) + 1
        sub = ch.take(np.flatnonzero(inband[key]))
        for ci, cond in enumerate(wl.conditions):
            Q, _ = oracle.partition(wl.states, wl.population, cond.T, cond.T_vib, cond.T_rot)
            nu_s, S_s, _ = oracle.intensities(wl.states, sub, wl.mode, wl.population, cond.T, Q,
                                              cond.T_vib, cond.T_rot)
            for b in bands:
                m = np.flatnonzero((nu_s >= b) & (nu_s < b + BAND_CM))
                top = m[np.argsort(S_s[m])[-STRONG:]]
                cand[ci].append((b, nu_s[top], S_s[top]))
    per = int(round(BAND_CM / wl.grid.dnu))
    bins = []
    for ci in range(len(wl.conditions)):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([5009, ci])))
        pts = []
        for b in bands:
            nus = np.concatenate([c[1] for c in cand[ci] if c[0] == b])
            Ss = np.concatenate([c[2] for c in cand[ci] if c[0] == b])
            best = nus[np.argsort(Ss)[-STRONG:]]
            kc = np.rint((best - wl.grid.nu0) / wl.grid.dnu).astype(np.int64)
            pts.append((kc[:, None] + OFFSETS[None, :]).ravel())
            k0 = int(round((b - wl.grid.nu0) / wl.grid.dnu))
            pts.append(k0 + rng.integers(0, per, UNIFORM))
        bb = np.unique(np.concatenate(pts))
        bins.append(bb[(bb >= 0) & (bb < wl.grid.n_bins)])
    return bins


def test_streamed_1e9_lines_full_size(stream1e9):
    wl, chunks, out = stream1e9
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(5009)))
    bands = rng.integers(100, 30000 - BAND_CM - 100, BANDS)
    bins = _strong_and_points(wl, chunks, bands)
    cut = max(c.cutoff for c in wl.conditions)
    # 1 cm^-1 buckets (index b + 1 holds wavenumbers in [b, b + 1)) within
    # cut + 2 cm^-1 of any sampled point
    nb = int(np.ceil(wl.grid.nu0 + wl.grid.n_bins * wl.grid.dnu)) + 3
    want = np.zeros(nb + 1, bool)
    for k in np.unique(np.concatenate(bins)):
        nu_k = wl.grid.nu0 + k * wl.grid.dnu
        lo = max(int(np.floor(nu_k - cut)) - 2, -1)
        hi = min(int(np.floor(nu_k + cut)) + 2, nb - 1)
        want[lo + 1:hi + 2] = True
    E = wl.states.energy
    parts = []
    for j, ch in enumerate(chunks):
        nu = E[ch.upper] - E[ch.lower]
        key = np.clip(np.floor(nu), -1, nb - 1).astype(np.int32) + 1
        parts.append(ch.take(np.flatnonzero(want[key])))
    sub = synth.Lines(np.concatenate([p.upper for p in parts]), np.concatenate([p.lower for p in parts]),
                      np.concatenate([p.einstein_a for p in parts]), None, None,
                      chunks[0].gamma_ref_scalar, chunks[0].n_exp_scalar)
    log(f"[stream1e9] {sub.n} lines near the sampled points")
    n_total = 0
    for ci, cond in enumerate(wl.conditions):
        ref = oracle.run_condition(wl, sub, cond, bins=bins[ci]).sigma
        s64, s32 = out["f64"][ci], out["f32"][ci]
        peak = float(ref.max())
        for name, got, tol in (("fp64", s64, 1e-10), ("fp32", s32, 1e-4)):
            e, l1, n = rel_err(got[bins[ci]], ref, peak=peak)
            log(f"[stream1e9] Tv={cond.T_vib:g} Tr={cond.T_rot:g} {name}: max_rel={e:.2e} over {n} of "
                f"{len(bins[ci])} points")
            assert n >= 50, (ci, name, n)
            assert e <= tol, (ci, name, e)
        n_total += n
    assert n_total >= 400
