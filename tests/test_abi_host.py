"""The C-ABI on the host, without a GPU: the shared library loads and exports
every function that include/xsec.h declares; the Python binding's structs have
the header's layout (checked against a C program compiled from the header);
host-side validation rejects bad arguments with XS_EINVAL before any GPU call;
and the binding fails loudly when the library is missing."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xsec.h")


def _binding():
    import paper_2609_17273_amd.xsec as X
    if not os.path.exists(X.LIB_PATH):
        pytest.skip("libxsec.so is not built (run __graft_entry__.build())")
    return X


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(xs_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_names():
    X = _binding()
    names = _declared_functions()
    assert len(names) >= 20
    assert names == sorted(X.SIGNATURES), (set(names) ^ set(X.SIGNATURES))


def test_library_exports_every_declared_symbol(no_gpu_in_process):
    X = _binding()
    lib = C.CDLL(X.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and nm agrees that they are exported, global text symbols
    out = subprocess.run(["nm", "-D", "--defined-only", X.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(_declared_functions()) <= exported
    assert X.lib().xs_version().decode().startswith("xsec")


_STRUCTS = {
    "xs_model": ["profile", "mode", "population", "precision", "algo", "mass_amu", "T_ref", "P_ref",
                 "hwhm_fixed"],
    "xs_grid": ["nu0", "dnu", "n_bins"],
    "xs_condition": ["T", "P", "T_vib", "T_rot", "cutoff"],
    "xs_states": ["n", "energy", "g_tot", "v", "e_vib", "n_v", "n_vib", "lifetime"],
    "xs_lines": ["n", "upper", "lower", "einstein_a", "gamma_ref", "n_exp", "log_scale",
                 "gamma_ref_scalar", "n_exp_scalar"],
    "xs_config": ["tile_bins", "bucket_bins", "persistent", "waves_per_cu", "chunk_lines", "adj_blocks"],
    "xs_stats": ["lines_in", "lines_kept", "window_pairs", "work_items", "lines_invalid"],
}


def test_struct_layout_matches_header(tmp_path, no_gpu_in_process):
    X = _binding()
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for s, fields in _STRUCTS.items():
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'  printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            parts = ln.split()
            got[(parts[0], parts[1])] = int(parts[2])
    for s, fields in _STRUCTS.items():
        cls = getattr(X, s)
        assert [f[0] for f in cls._fields_] == fields
        assert C.sizeof(cls) == got[(s, "size")], s
        for f in fields:
            assert getattr(cls, f).offset == got[(s, f)], (s, f)


def _model(X, **kw):
    m = X.xs_model(X.XS_VOIGT, X.XS_ABSORPTION, X.XS_LTE, X.XS_FP32, X.XS_GATHER, 30.0, 296.0, 1.0, 0.0)
    for k, v in kw.items():
        setattr(m, k, v)
    return m


def _create(X, model=None, grid=None, conds=None, max_lines=100):
    model = model or _model(X)
    grid = grid or X.xs_grid(0.0, 0.01, 1001)
    conds = conds if conds is not None else [X.xs_condition(1000.0, 1.0, 1000.0, 1000.0, 25.0)]
    arr = (X.xs_condition * max(1, len(conds)))(*conds)
    out = C.c_void_p()
    rc = X.lib().xs_plan_create(C.byref(out), C.byref(model), C.byref(grid), len(conds), arr, max_lines, None)
    return rc, X.lib().xs_last_error().decode()


@pytest.mark.parametrize("case", [
    "profile", "mode", "population", "precision", "algo", "mass", "T_ref", "P_ref", "hwhm",
    "dnu", "nu0", "n_bins", "n_cond", "cutoff", "T", "P", "lorentz_P0", "Tvib", "max_lines",
    "bin_hwhm", "bin_mass", "bin_lorentz_P0", "profile_neg", "density_Trot0"])
def test_plan_create_rejects_bad_arguments(case):
    X = _binding()
    nan = float("nan")
    cond = lambda **kw: X.xs_condition(kw.get("T", 1000.0), kw.get("P", 1.0), kw.get("Tv", 1000.0),
                                       kw.get("Tr", 1000.0), kw.get("cut", 25.0))
    args = {
        "profile": dict(model=_model(X, profile=10)),
        "mode": dict(model=_model(X, mode=-1)),
        "population": dict(model=_model(X, population=5)),
        "precision": dict(model=_model(X, precision=2)),
        "algo": dict(model=_model(X, algo=3)),
        "mass": dict(model=_model(X, mass_amu=0.0)),
        "T_ref": dict(model=_model(X, T_ref=-1.0)),
        "P_ref": dict(model=_model(X, P_ref=nan)),
        "hwhm": dict(model=_model(X, profile=X.XS_GAUSSIAN, hwhm_fixed=0.0)),
        "dnu": dict(grid=X.xs_grid(0.0, 0.0, 100)),
        "nu0": dict(grid=X.xs_grid(float("inf"), 0.01, 100)),
        "n_bins": dict(grid=X.xs_grid(0.0, 0.01, 0)),
        "n_cond": dict(conds=[]),
        "cutoff": dict(conds=[cond(cut=0.0)]),
        "T": dict(conds=[cond(T=0.0)]),
        "P": dict(conds=[cond(P=-1.0)]),
        "lorentz_P0": dict(model=_model(X, profile=X.XS_LORENTZ), conds=[cond(P=0.0)]),
        "Tvib": dict(model=_model(X, population=X.XS_NLTE_2T), conds=[cond(Tv=0.0)]),
        "max_lines": dict(max_lines=0),
        "bin_hwhm": dict(model=_model(X, profile=X.XS_BIN_GAUSSIAN, hwhm_fixed=-1.0)),
        "bin_mass": dict(model=_model(X, profile=X.XS_BIN_VOIGT, mass_amu=0.0)),
        "bin_lorentz_P0": dict(model=_model(X, profile=X.XS_BIN_LORENTZ), conds=[cond(P=0.0)]),
        "profile_neg": dict(model=_model(X, profile=-1)),
        "density_Trot0": dict(model=_model(X, population=X.XS_NLTE_DENSITY), conds=[cond(Tr=0.0)]),
    }[case]
    rc, msg = _create(X, **args)
    assert rc == X.XS_EINVAL, (case, rc, msg)
    assert msg, case


def test_null_plan_and_null_out_are_errors():
    X = _binding()
    L = X.lib()
    m, g = _model(X), X.xs_grid(0.0, 0.01, 10)
    c = (X.xs_condition * 1)(X.xs_condition(1000.0, 1.0, 1000.0, 1000.0, 25.0))
    assert L.xs_plan_create(None, C.byref(m), C.byref(g), 1, c, 10, None) == X.XS_EINVAL
    assert L.xs_plan_replay(None) == X.XS_EINVAL
    assert L.xs_plan_sync(None) == X.XS_EINVAL
    assert L.xs_plan_set_config(None, None) == X.XS_EINVAL
    assert L.xs_profile_pass(None, None, 0) == X.XS_EINVAL
    n = C.c_size_t()
    assert L.xs_plan_workspace_bytes(None, C.byref(n)) == X.XS_EINVAL
    L.xs_plan_destroy(None)  # a no-op


def test_binding_fails_loudly_without_the_library(monkeypatch):
    import paper_2609_17273_amd.xsec as X
    monkeypatch.setattr(X, "_lib", None)
    monkeypatch.setattr(X, "LIB_PATH", "/nonexistent/libxsec.so")
    with pytest.raises(RuntimeError, match="missing"):
        X.lib()
