"""The seeded input generator: determinism, ranges and distributions of the
synthetic stand-ins for the paper's line lists."""
import numpy as np

import synth


def test_deterministic_per_seed_and_chunk():
    a = synth.workload("voigt_1e7", n_states=5000, n_lines=20000)
    b = synth.workload("voigt_1e7", n_states=5000, n_lines=20000)
    np.testing.assert_array_equal(a.states.energy, b.states.energy)
    la, lb = a.lines(), b.lines()
    for f in ("upper", "lower", "einstein_a", "gamma_ref", "n_exp"):
        np.testing.assert_array_equal(getattr(la, f), getattr(lb, f))
    c = synth.workload("twotemp_1e9", n_states=3000, n_lines=40000, n_chunks=4)
    np.testing.assert_array_equal(c.chunk(2).upper, c.chunk(2).upper)
    assert not np.array_equal(c.chunk(1).upper, c.chunk(2).upper)


def test_ranges_and_distributions():
    wl = synth.workload("voigt_1e7", n_states=20000, n_lines=100000)
    st, ln = wl.states, wl.lines()
    assert st.energy[0] == 0.0 and st.g_tot[0] == 1.0
    assert st.energy.max() <= 40000.0
    assert abs(st.energy[1:].mean() - 8000.0) < 300.0   # truncated exponential, mean ~7.7e3
    nu = st.energy[ln.upper] - st.energy[ln.lower]
    assert (nu > 0).all() and (nu <= 20000.0).all()
    assert (ln.upper != ln.lower).all()
    la = np.log10(ln.einstein_a.astype(np.float64))
    assert la.min() >= -8.0 - 1e-6 and la.max() <= 3.0 + 1e-6
    assert ln.einstein_a.dtype == np.float32 and ln.gamma_ref.dtype == np.float32
    assert 0.02 * (1 - 1e-6) <= ln.gamma_ref.min() and ln.gamma_ref.max() <= 0.1 * (1 + 1e-6)
    assert 0.3 <= ln.n_exp.min() and ln.n_exp.max() <= 0.8
    g = (st.g_tot - 1) / 2
    assert g.min() == 0 and g.max() == 120
    assert wl.grid.n_bins == 2_000_001 and wl.grid.dnu == 0.01


def test_two_temperature_states():
    wl = synth.workload("twotemp_1e9", n_states=10000, n_lines=1000, n_chunks=1)
    st = wl.states
    v = st.v
    assert v.min() == 0 and v.max() == 10
    J = (st.g_tot - 1) / 2
    np.testing.assert_array_equal(st.energy, st.e_vib[v] + J * (J + 1))
    assert st.e_vib[10] == 18900.0
    nu = st.energy[wl.lines().upper] - st.energy[wl.lines().lower]
    assert (nu > 0).all() and (nu <= 30000.0).all()
    assert len(wl.conditions) == 4 and wl.grid.n_bins == 600_001


def test_full_size_shapes_without_drawing_lines():
    assert synth.workload("voigt_grid48_1e8").n_lines == 100_000_000 and len(synth.workload("voigt_grid48_1e8").conditions) == 48
    tt = synth.workload("twotemp_1e9")
    assert tt.n_lines == 1_000_000_000 and tt.n_chunks == 10 and tt.chunk_sizes()[0] == 100_000_000
    assert [c.cutoff for c in synth.workload("voigt_grid48_1e8").conditions[:6]] == [25.0, 25.0, 25.0, 100.0, 100.0, 100.0]
