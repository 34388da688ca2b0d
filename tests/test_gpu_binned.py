"""Binned (bin-integrated) profiles on the GPU against the oracle.

The binned methods of Table tab:profile: sigma_k = sum_i S_i fbar_ik with
fbar the mean of the profile over the bin centred on grid point k, over the
same cut-off windows (bin centres within the cut-off).  Same bar as the
sampled profiles: max relative error over bins with sigma_ref >= 1e-6 of the
peak, 1e-10 (FP64 form) and 1e-4 (FP32 form).  Cases: binned Doppler (the
Doppler workload's width ~ the bin), fixed-HWHM Gaussian, Lorentzian, Voigt
at moderate pressure, at 1e-4 bar and 300 K (lines far narrower than a bin,
so each line's central bin holds nearly all of it) and at 100 bar (Lorentzian
widths of many bins), two-temperature emission; gather (three tile sizes,
persistent and not) and scatter; and the full 1e7-line Voigt workload at
sampled points.
"""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, gpu_inputs, gpu_sigma, log, make_plan, rel_err

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-10, FP32: 1e-4}


def _wl(name):
    if name == "doppler":
        return synth.workload("doppler_1e4", n_lines=3000, nu_hi=1500.0, profile=synth.BIN_DOPPLER)
    if name == "gaussian":
        wl = synth.workload("voigt_1e7", n_states=5000, n_lines=3000, nu_hi=400.0, profile=synth.BIN_GAUSSIAN)
        wl.hwhm_fixed = 0.037
        return wl
    if name == "lorentz":
        return synth.workload("voigt_1e7", n_states=20000, n_lines=3000, nu_hi=300.0, profile=synth.BIN_LORENTZ)
    if name == "voigt":
        return synth.workload("voigt_1e7", n_states=20000, n_lines=2000, nu_hi=250.0, profile=synth.BIN_VOIGT)
    if name == "voigt_lowP":
        return synth.workload("voigt_1e7", n_states=20000, n_lines=2000, nu_hi=250.0, profile=synth.BIN_VOIGT,
                            seed=1212, conditions=[synth.Condition(300.0, 1e-4, 25.0)])
    if name == "voigt_highP":
        return synth.workload("voigt_1e7", n_states=20000, n_lines=1500, nu_hi=250.0, profile=synth.BIN_VOIGT,
                            seed=1213, conditions=[synth.Condition(300.0, 100.0, 100.0)])
    if name == "em2T":
        return synth.workload("twotemp_1e9", n_states=20000, n_lines=6000, n_chunks=1, nu_hi=1500.0,
                            profile=synth.BIN_DOPPLER)
    raise KeyError(name)


NAMES = ["doppler", "gaussian", "lorentz", "voigt", "voigt_lowP", "voigt_highP", "em2T"]
_REF = {}


def _ref(name):
    if name not in _REF:
        wl = _wl(name)
        ln = wl.lines()
        _REF[name] = [oracle.run_condition(wl, ln, c).sigma for c in wl.conditions]
    return _REF[name]


def _check(tag, got, ref, prec, st=None):
    e, l1, n = rel_err(got, ref)
    log(f"[binned {tag}] prec={'fp32' if prec else 'fp64'} max_rel={e:.3e} L1={l1:.3e} bins={n}"
        + (f" stats={st}" if st else ""))
    assert n > 0
    assert e <= TOL[prec], f"{tag}: {e} > {TOL[prec]}"
    assert np.all(got[ref == 0.0] == 0.0)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_binned_gather_small(name, prec):
    wl = _wl(name)
    ref = _ref(name)
    got, st, _ = gpu_sigma(wl, wl.lines(), prec)
    for c in range(len(wl.conditions)):
        _check(f"{name}/c{c}", got[c], ref[c], prec, st if c == 0 else None)


@pytest.mark.parametrize("name", ["doppler", "lorentz", "voigt", "voigt_lowP"])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_binned_scatter_small(name, prec):
    wl = _wl(name)
    ref = _ref(name)
    got, st, _ = gpu_sigma(wl, wl.lines(), prec, algo=1)
    _check(f"{name}/scatter", got[0], ref[0], prec)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_binned_voigt_tile_configs(prec):
    wl = _wl("voigt")
    ref = _ref("voigt")[0]
    for tile in (256, 512, 1024):
        for persistent in (0, 1):
            cfg = dict(tile_bins=tile, persistent=persistent, waves_per_cu=16, chunk_lines=0)
            got, st, _ = gpu_sigma(wl, wl.lines(), prec, config=cfg)
            _check(f"voigt/tile{tile}/p{persistent}", got[0], ref, prec)


def test_binned_adjoint_unsupported():
    import torch
    P = X()
    wl = _wl("voigt")
    ln = wl.lines()
    plan = make_plan(wl, FP32, ln.n)
    ds, dl = gpu_inputs(wl, ln)
    g = torch.zeros((1, wl.grid.n_bins), dtype=torch.float64, device="cuda")
    with pytest.raises(P.XsecError) as ei:
        plan.adjoint(ds, dl, g)
    assert ei.value.code == P.XS_EUNSUPPORTED
    plan.close()


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_binned_voigt_full_size_sampled(prec):
    wl = synth.workload("voigt_1e7", profile=synth.BIN_VOIGT)
    ln = wl.lines()
    got, st, dt = gpu_sigma(wl, ln, prec)
    got = got[0]
    cond = wl.conditions[0]
    r0 = oracle.run_condition(wl, ln, cond, with_sigma=False)
    top = np.argsort(r0.S)[-150:]
    kc = np.rint((r0.nu[top] - wl.grid.nu0) / wl.grid.dnu).astype(np.int64)
    near = (kc[:, None] + np.array([-2, 0, 1, 5])[None, :]).ravel()
    near = near[(near >= 0) & (near < wl.grid.n_bins)]
    bins = np.unique(np.concatenate([synth.sample_bins(wl.grid.n_bins, 1500, 91), near,
                                     [int(np.argmax(got))]]))
    ref = oracle.run_condition(wl, ln, cond, bins=bins).sigma
    peak = max(float(ref.max()), float(got.max()))
    e, l1, n = rel_err(got[bins], ref, peak=peak)
    log(f"[binned full] prec={prec} max_rel={e:.3e} L1={l1:.3e} over {n} sampled points; {st}")
    assert n > 500
    assert e <= TOL[prec]


@pytest.mark.parametrize("hwhm", [0.002, 0.3])
@pytest.mark.parametrize("tile", [256, 1024])
def test_binned_gaussian_widths(hwhm, tile):
    """Fixed-width binned Gaussian at step 0.01 with a few nonzero bins per
    line (one line per lane) and with more than a tile of them (whole-row
    and 64-point wave steps)."""
    wl = synth.workload("voigt_1e7", n_states=5000, n_lines=3000, nu_hi=400.0, profile=synth.BIN_GAUSSIAN)
    wl.hwhm_fixed = hwhm
    ln = wl.lines()
    ref = oracle.run_condition(wl, ln, wl.conditions[0]).sigma
    for prec in (FP64, FP32):
        got, st, _ = gpu_sigma(wl, ln, prec, config=dict(tile_bins=tile, bucket_bins=64, persistent=1,
                                                         waves_per_cu=16))
        _check(f"gaussian hwhm={hwhm} tile={tile}", got[0], ref, prec, st)
