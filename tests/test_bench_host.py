"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the Voigt region
fractions behind the flop counts, and the traffic and VALU figures' source
check."""
import json
import os
import subprocess
import sys

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused(no_gpu_in_process):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_region_fractions_partition_the_evaluations():
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=20000, nu_hi=5000.0)
    ln = wl.lines()
    fr = bench.region_fractions(wl, ln, wl.conditions[0])
    for kind, f in fr.items():
        assert len(f) == len(bench.FLOP_REGIONS[kind])
        assert all(x >= 0.0 for x in f)
        assert abs(sum(f) - 1.0) < 1e-12, kind
    # the same thresholds give the same split in both forms' outer regions
    assert fr[("fwd", "f32")] == fr[("adj", "f32")]


def test_region_fractions_match_a_brute_force_count():
    """The closed form against counting |x|^2 + y^2 per grid point of the
    windows of a few lines (grid clipping excluded: lines in the middle)."""
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=40, nu_hi=3000.0)
    ln = wl.lines()
    cond = wl.conditions[0]
    E = wl.states.energy
    nu = E[ln.upper] - E[ln.lower]
    keep = (nu > 100.0) & (nu < 2900.0)
    ln = ln.take(np.flatnonzero(keep))
    nu = nu[keep]
    fr = bench.region_fractions(wl, ln, cond)[("fwd", "f32")]
    c, kb, amu = 2.99792458e10, 1.380649e-16, 1.66053906660e-24
    alpha = nu / c * np.sqrt(2.0 * kb * cond.T * np.log(2.0) / (wl.mass_amu * amu))
    s = alpha / np.sqrt(np.log(2.0))
    y = ln.gamma_ref.astype(np.float64) * (296.0 / cond.T) ** ln.n_exp.astype(np.float64) * cond.P / s
    counts = np.zeros(3)
    step = 1e-3
    for i in range(len(nu)):
        d = np.arange(-cond.cutoff, cond.cutoff, step)
        rho = (d / s[i]) ** 2 + y[i] ** 2
        counts += [np.sum(rho >= 900.0), np.sum((rho < 900.0) & (rho >= 64.0)), np.sum(rho < 64.0)]
    brute = counts / counts.sum()
    assert np.allclose(fr, brute, atol=2e-4), (fr, brute)


def test_traffic_only_for_the_current_sources():
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    with open(path) as f:
        d = json.load(f)
    for key in ("gather_voigt1e7_f32", "adjoint_voigt1e7_f32"):
        got = bench.traffic_from_profiles(key)
        if d[key]["source_hash"] == bench.source_hash():
            assert got == d[key]["hbm_bytes_per_launch"] and got > 0
        else:
            assert got is None


def test_valu_issue_only_for_the_current_sources():
    """The VALU issue figures: None when the counters were taken on other
    sources; otherwise wave instructions x 4 cycles over 1024 SIMDs x 2.4 GHz
    x time (the sampled clock is only reported), and lane instructions per
    evaluation."""
    path = os.path.join(ROOT, "profiles", "pmc_valu.json")
    with open(path) as f:
        d = json.load(f)
    for key in ("gather_voigt1e7_f32", "adjoint_voigt1e7_f64"):
        got = bench.valu_from_profiles(key, 10.0, 2250.0)
        e = d[key]
        if e["source_hash"] != bench.source_hash():
            assert got is None
            continue
        n = e["SQ_INSTS_VALU"]
        assert got["wave_instructions"] == n
        assert abs(got["issue_frac"] - 4.0 * n / (1024 * 2.4e9 * 0.010)) < 1e-4
        assert abs(got["per_eval"] - n * 64 / e["evals"]) < 1e-3
        assert got["sclk_MHz_sampled"] == 2250.0


def test_adjoint_block_share_limits():
    """The share of adjoint waves in a block-summed form: all of them at a
    vanishing pressure, none at a huge one, and falling as y grows with P;
    the flop average moves between the two forms with it."""
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=5000, nu_hi=3000.0)
    ln = wl.lines()
    share = [bench.adj_block_share(wl, ln, synth.Condition(2000.0, P, 25.0), 450.0) for P in (1e-6, 0.3, 3.0, 1e4)]
    assert share[0] == 1.0 and share[-1] == 0.0
    assert share[0] >= share[1] >= share[2] >= share[3]
    assert 0.0 < share[1] < 1.0
    cond = wl.conditions[0]
    sh = bench.adj_block_shares(wl, ln, cond)
    assert len(sh) == 2 and sh[0] >= sh[1]    # the inner region asks for a smaller y
    fr = bench.region_fractions(wl, ln, cond)
    k = ("adj", "f32")
    lo, hi = bench.flops_per_eval(fr, k, [1.0, 1.0]), bench.flops_per_eval(fr, k, [0.0, 0.0])
    assert lo == bench.flops_per_eval(fr, k)
    want = sum(f * (pt - bl) for f, pt, bl in zip(fr[k], bench.ADJ_POINT_FLOPS["f32"],
                                                  [x for _, x in bench.FLOP_REGIONS[k]]))
    assert abs((hi - lo) - want) < 1e-12
