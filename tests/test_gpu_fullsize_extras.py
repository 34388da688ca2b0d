"""Parity of the benchmark's extra profile passes at their full size, in the
kernel configuration the benchmark's step uses (256-point tiles, persistent
launch): the 1e7-line Voigt workload (1e6 states, T 2000 K, P 1 bar, grid
0-20000 cm^-1 step 0.01, cut-off 25 cm^-1) with the Olivero and Thompson
pseudo-Voigts, and with predissociation lifetimes on a third of the states
(Voigt), FP32 form.

sigma is checked at sampled points, which the oracle computes one by one over
all 1e7 lines: 1,500 random points, points near the 150 strongest lines and
the peak.
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import gpu_sigma, log, rel_err

pytestmark = pytest.mark.gpu
FP32 = 1
CFG = dict(tile_bins=256, bucket_bins=256, persistent=1, waves_per_cu=16)


def _sampled(wl, ln, got, seed):
    cond = wl.conditions[0]
    r0 = oracle.run_condition(wl, ln, cond, with_sigma=False)
    top = np.argsort(r0.S)[-150:]
    kc = np.rint((r0.nu[top] - wl.grid.nu0) / wl.grid.dnu).astype(np.int64)
    near = (kc[:, None] + np.array([-3, 0, 1, 7])[None, :]).ravel()
    near = near[(near >= 0) & (near < wl.grid.n_bins)]
    bins = np.unique(np.concatenate([synth.sample_bins(wl.grid.n_bins, 1500, seed), near,
                                     [int(np.argmax(got))]]))
    ref = oracle.run_condition(wl, ln, cond, bins=bins).sigma
    peak = max(float(ref.max()), float(got.max()))
    return rel_err(got[bins], ref, peak=peak)


@pytest.mark.parametrize("kind", [synth.PV_OLIVERO, synth.PV_THOMPSON])
def test_pseudo_voigt_full_size_sampled(kind):
    wl = synth.workload("voigt_1e7", profile=kind)
    ln = wl.lines()
    got, st, _ = gpu_sigma(wl, ln, FP32, config=CFG)
    e, l1, n = _sampled(wl, ln, got[0], 93)
    log(f"[pv full] kind={kind} max_rel={e:.3e} L1={l1:.3e} over {n} sampled points")
    assert n > 400
    assert e <= 1e-4


def test_lifetime_voigt_full_size_sampled():
    wl = synth.workload("voigt_1e7")
    synth.with_lifetimes(wl, frac=0.33, seed=5)
    ln = wl.lines()
    got, st, _ = gpu_sigma(wl, ln, FP32, config=CFG)
    e, l1, n = _sampled(wl, ln, got[0], 95)
    log(f"[lifetime full] max_rel={e:.3e} L1={l1:.3e} over {n} sampled points")
    assert n > 400
    assert e <= 1e-4
