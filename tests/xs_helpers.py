"""Shared helpers of the GPU tests: run the HIP path through the C-ABI binding
and the oracle on the same seeded inputs, and compare them."""
from __future__ import annotations

import functools
import sys
import time
from typing import Optional

import numpy as np

import oracle
import synth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got: np.ndarray, ref: np.ndarray, peak: Optional[float] = None, thr: float = 1e-6):
    """Max relative error over bins with ref >= thr * peak, and the paper's
    normalised L1 error sum|got - ref| / sum|ref| (Eq. profile_gpu_error)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    peak = float(np.max(np.abs(ref))) if peak is None else peak
    m = np.abs(ref) >= thr * peak
    if not m.any():
        return 0.0, 0.0, 0
    e = float(np.max(np.abs(got[m] - ref[m]) / np.abs(ref[m])))
    l1 = float(np.sum(np.abs(got - ref)) / max(np.sum(np.abs(ref)), 1e-300))
    return e, l1, int(m.sum())


def X():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU")
    import paper_2609_17273_amd as P
    P.lib()
    return P


def gpu_inputs(wl, lines, log_scale=None):
    P = X()
    return P.DeviceStates.from_numpy(wl.states), P.DeviceLines.from_numpy(lines, log_scale=log_scale)


def make_plan(wl, precision, max_lines, algo=0, conditions=None):
    P = X()
    return P.Plan(wl.profile, wl.mode, wl.population, precision, wl.grid,
                  conditions if conditions is not None else wl.conditions, max_lines,
                  mass_amu=wl.mass_amu, algo=algo, T_ref=wl.T_ref, P_ref=wl.P_ref,
                  hwhm_fixed=wl.hwhm_fixed)


def gpu_sigma(wl, lines, precision, algo=0, config=None, log_scale=None):
    import torch
    plan = make_plan(wl, precision, max(lines.n, 1), algo)
    if config:
        plan.set_config(**config)
    ds, dl = gpu_inputs(wl, lines, log_scale)
    t0 = time.time()
    sig = plan.cross_section(ds, dl)
    torch.cuda.synchronize()
    st = plan.stats()
    out = sig.cpu().numpy()
    plan.close()
    return out, st, time.time() - t0


@functools.lru_cache(maxsize=16)
def _cached_workload(key):
    k, kw = key
    return synth.workload(k, **dict(kw))


def workload(k, **kw):
    return _cached_workload((k, tuple(sorted(kw.items()))))


@functools.lru_cache(maxsize=32)
def _oracle_sigma(key, ci, bins_key):
    k, kw = key
    wl = _cached_workload(key)
    bins = None if bins_key is None else np.frombuffer(bins_key, dtype=np.int64)
    r = oracle.run_condition(wl, wl.lines(), wl.conditions[ci], bins=bins)
    return r.sigma


def oracle_sigma(wl_key_k, wl_kw, ci=0, bins=None):
    key = (wl_key_k, tuple(sorted(wl_kw.items())))
    return _oracle_sigma(key, ci, None if bins is None else np.ascontiguousarray(bins, np.int64).tobytes())


def check_line_gradients(tag, got, ref, bound, tol, thr=1e-6):
    """Per-line adjoint gradients (one vector) against the oracle's.

    * ||got - ref||_2 / ||ref||_2 <= tol;
    * per element, relative to the sum's own scale: |got_i - ref_i| <= tol
      bound_i, with bound_i the same gradient with every term of its window
      sum taken in absolute value (``oracle.adjoint_bounds``), over the
      elements with bound_i >= thr max(bound).  A per-line gradient is a
      signed sum over its window (cotangents of either sign, profile
      derivatives that change sign) that can cancel to any degree, so its
      error is measured against what rounding in its terms can move it by;
    * per element, the plain relative error |got_i - ref_i| / |ref_i| over
      the elements with |ref_i| >= thr max|ref|: logged (largest, and 99.9th
      percentile), and asserted <= tol over those whose sum does not cancel
      (bound_i <= 2 |ref_i|; every element when the terms share one sign).
    Returns the componentwise error."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    bound = np.asarray(bound, np.float64)
    assert np.all(bound >= np.abs(ref) * (1 - 1e-12)), tag  # the oracle's own consistency
    e_norm = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    mb = bound >= thr * float(bound.max()) if bound.size else bound.astype(bool)
    e_comp = float(np.max(np.abs(got[mb] - ref[mb]) / bound[mb])) if mb.any() else 0.0
    mr = np.abs(ref) >= thr * float(np.abs(ref).max()) if ref.size else ref.astype(bool)
    rel = np.abs(got[mr] - ref[mr]) / np.abs(ref[mr]) if mr.any() else np.zeros(0)
    well = mr & (bound <= 2.0 * np.abs(ref))
    e_well = float(np.max(np.abs(got[well] - ref[well]) / np.abs(ref[well]))) if well.any() else 0.0
    log(f"[grad] {tag}: norm {e_norm:.2e}; componentwise {e_comp:.2e} over {int(mb.sum())}; "
        f"relative max {float(rel.max()) if rel.size else 0.0:.2e} "
        f"p99.9 {float(np.quantile(rel, 0.999)) if rel.size else 0.0:.2e} over {int(mr.sum())}; "
        f"well-conditioned {e_well:.2e} over {int(well.sum())}")
    assert e_norm <= tol, (tag, "norm", e_norm)
    assert e_comp <= tol, (tag, "componentwise", e_comp)
    assert e_well <= tol, (tag, "relative (well-conditioned)", e_well)
    # no element the oracle leaves at exactly zero (no window) gets a value
    assert np.all(got[bound == 0.0] == 0.0), tag
    return e_comp
