"""FP64 CPU oracle for the line-list cross-section path.

TEST INFRASTRUCTURE ONLY: tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(``paper_2609_17273_amd``) never imports this package, and this package never
imports the product: the two share only the seeded input generator ``synth``.

The arithmetic lives in ``xsec_oracle.c`` (plain C, FP64, no FMA contraction,
OpenMP over independent bins or lines); this module marshals numpy arrays into
it and assembles the adjoint's chain rule (numpy, FP64).  Each step cites the
paper passage it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xsec_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
           "-std=gnu11"]

DOPPLER, GAUSSIAN, LORENTZ, VOIGT = 0, 1, 2, 3
# bin-integrated forms: the mean of the profile over the bin centred on the point
BIN_DOPPLER, BIN_GAUSSIAN, BIN_LORENTZ, BIN_VOIGT = 4, 5, 6, 7
# pseudo-Voigt approximations (widths of the Voigt)
PV_THOMPSON, PV_OLIVERO = 8, 9
ABSORPTION, EMISSION = 0, 1
LTE, NLTE_2T, NLTE_DENSITY = 0, 1, 2


def _stale() -> bool:
    return not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (it is test infrastructure, built in-tree).

    This starts a child process, so callers run it before their process
    touches the GPU (the test session's configure hook, the start of
    ``bench.py`` and ``smoke()``): a process that has initialised the GPU must
    not start other programs."""
    if force or _stale():
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    """Load the built oracle.  Never compiles: a missing or stale library
    raises (build it with ``build()`` before any GPU work)."""
    global _lib
    if _lib is None:
        if _stale():
            raise RuntimeError(f"{_LIB} is missing or older than {_SRC}: call oracle.build() "
                               "before the process uses the GPU")
        L = C.CDLL(_LIB)
        d, i64, i32, p = C.c_double, C.c_int64, C.c_int, C.c_void_p
        L.or_c2.restype = d
        L.or_max_threads.restype = i32
        L.or_set_threads.argtypes = [i32]
        L.or_set_threads.restype = None
        L.or_constants.argtypes = [p]
        L.or_partition.argtypes = [i64, p, p, p, p, p, i32, d, d, d, p, p]
        L.or_intensities.argtypes = [i64, p, p, p, p, p, p, p, p, p, i32, i32, d, d, d, d, p, p, p]
        L.or_dlnS_dT.argtypes = [i64, p, p, p, i32, d, d, d, p]
        L.or_cooling.argtypes = [i64, p, p, p, i64, p, p, i32, p, p, p]
        L.or_widths.argtypes = [i64, p, p, p, d, d, i32, d, d, d, d, d, d, p, p, p, p]
        L.or_faddeeva.argtypes = [d, d, p, p]
        L.or_faddeeva_deriv.argtypes = [d, d, p, p, p, p]
        L.or_profile.argtypes = [i32, d, d, d]
        L.or_profile.restype = d
        L.or_binned.argtypes = [i32, d, d, d, d]
        L.or_binned.restype = d
        L.or_gl_rule.argtypes = [p, p]
        L.or_window_counts.argtypes = [i64, p, d, d, d, i64, p]
        L.or_window_counts.restype = i64
        L.or_sigma.argtypes = [i64, p, p, p, p, i32, d, d, i64, d, i64, p, p]
        L.or_adjoint_sums.argtypes = [i64, p, p, p, i32, d, d, i64, d, p, p, p, p]
        L.or_adjoint_abs_sums.argtypes = [i64, p, p, p, i32, d, d, i64, d, p, p, p, p]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def c2() -> float:
    return lib().or_c2()


def constants() -> np.ndarray:
    """(h, c, k_B, amu, c2) as used by the oracle."""
    out = np.zeros(5)
    lib().or_constants(_p(out))
    return out


def threads() -> int:
    return lib().or_max_threads()


def set_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops (timing only)."""
    lib().or_set_threads(int(n))


def faddeeva(x: float, y: float) -> complex:
    re, im = C.c_double(), C.c_double()
    lib().or_faddeeva(float(x), float(y), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def faddeeva_deriv(x: float, y: float):
    """(w'(z), G(z) = w + z w') from the oracle's quadrature."""
    v = [C.c_double() for _ in range(4)]
    lib().or_faddeeva_deriv(float(x), float(y), *[C.byref(q) for q in v])
    return complex(v[0].value, v[1].value), complex(v[2].value, v[3].value)


def profile(kind: int, d: float, alpha: float, gamma: float) -> float:
    return lib().or_profile(int(kind), float(d), float(alpha), float(gamma))


def binned(kind: int, d: float, dnu: float, alpha: float, gamma: float) -> float:
    """Mean of the profile over [d - dnu/2, d + dnu/2] (kind: BIN_* or the sampled kind)."""
    return lib().or_binned(int(kind), float(d), float(dnu), float(alpha), float(gamma))


def gl_rule():
    """(nodes, weights) of the oracle's 16-point Gauss-Legendre rule on [-1, 1]."""
    x, w = np.empty(16), np.empty(16)
    lib().or_gl_rule(_p(x), _p(w))
    return x, w


def partition(states, pop: int, T: float, T_vib: float = 0.0, T_rot: float = 0.0):
    """(Q, dQ/dT) for one condition; dQ/dT is NaN for two temperatures."""
    E = _c(states.energy, np.float64)
    g = _c(states.g_tot, np.float64)
    v = _c(states.v, np.int32)
    ev = _c(states.e_vib, np.float64)
    nv = _c(getattr(states, "n_vib", None), np.float64)
    if pop == NLTE_DENSITY and nv is None:
        raise ValueError("custom vibronic densities need states.n_vib")
    Q, dQ = C.c_double(), C.c_double()
    lib().or_partition(E.shape[0], _p(E), _p(g), _p(v), _p(ev), _p(nv), pop, T, T_vib, T_rot,
                       C.byref(Q), C.byref(dQ))
    return Q.value, dQ.value


def intensities(states, lines, mode: int, pop: int, T: float, Q: float, T_vib: float = 0.0,
                T_rot: float = 0.0, log_scale: Optional[np.ndarray] = None):
    """(nu, S, keep) for every line (S = 0 and keep = 0 where nu <= 0)."""
    n = lines.n
    up = _c(lines.upper, np.int32)
    lo = _c(lines.lower, np.int32)
    A = _c(lines.einstein_a, np.float32)
    ls = _c(log_scale, np.float32)
    E = _c(states.energy, np.float64)
    g = _c(states.g_tot, np.float64)
    v = _c(states.v, np.int32)
    ev = _c(states.e_vib, np.float64)
    nv = _c(getattr(states, "n_vib", None), np.float64)
    if pop == NLTE_DENSITY and nv is None:
        raise ValueError("custom vibronic densities need states.n_vib")
    nu = np.empty(n)
    S = np.empty(n)
    keep = np.empty(n, np.int8)
    lib().or_intensities(n, _p(up), _p(lo), _p(A), _p(ls), _p(E), _p(g), _p(v), _p(ev), _p(nv),
                         mode, pop, T, T_vib, T_rot, Q, _p(nu), _p(S), _p(keep))
    return nu, S, keep


def cooling(states, lines, T) -> tuple:
    """(W(T), Q(T)) at the temperatures T (Eq. cf), erg s^-1 molecule^-1 sr^-1."""
    T = _c(np.atleast_1d(T), np.float64)
    up = _c(lines.upper, np.int32)
    lo = _c(lines.lower, np.int32)
    A = _c(lines.einstein_a, np.float32)
    E = _c(states.energy, np.float64)
    g = _c(states.g_tot, np.float64)
    W = np.empty(T.shape[0])
    Q = np.empty(T.shape[0])
    lib().or_cooling(lines.n, _p(up), _p(lo), _p(A), E.shape[0], _p(E), _p(g), T.shape[0], _p(T),
                     _p(W), _p(Q))
    return W, Q


def dlnS_dT(states, lines, mode: int, T: float, Q: float, dQdT: float) -> np.ndarray:
    out = np.empty(lines.n)
    up = _c(lines.upper, np.int32)
    lo = _c(lines.lower, np.int32)
    E = _c(states.energy, np.float64)
    lib().or_dlnS_dT(lines.n, _p(up), _p(lo), _p(E), mode, T, Q, dQdT, _p(out))
    return out


def widths(nu, lines, prof: int, T: float, P: float, mass_amu: float, T_ref: float = 296.0,
           P_ref: float = 1.0, hwhm_fixed: float = 0.0, lifetime: Optional[np.ndarray] = None):
    """(alpha, gamma) per line; ``lifetime`` (per state, s) adds the upper
    state's natural width to gamma."""
    n = nu.shape[0]
    nu = _c(nu, np.float64)
    gr = _c(lines.gamma_ref, np.float32)
    ne = _c(lines.n_exp, np.float32)
    tau = _c(lifetime, np.float64)
    up = _c(lines.upper, np.int32) if lifetime is not None else None
    alpha = np.empty(n)
    gamma = np.empty(n)
    lib().or_widths(n, _p(nu), _p(gr), _p(ne), float(lines.gamma_ref_scalar),
                    float(lines.n_exp_scalar), prof, T, P, mass_amu, T_ref, P_ref,
                    hwhm_fixed, _p(tau), _p(up), _p(alpha), _p(gamma))
    return alpha, gamma


def window_counts(nu, cut: float, grid):
    nu = _c(nu, np.float64)
    counts = np.empty(nu.shape[0], np.int64)
    tot = lib().or_window_counts(nu.shape[0], _p(nu), cut, grid.nu0, grid.dnu, grid.n_bins,
                                 _p(counts))
    return tot, counts


def sigma(nu, S, alpha, gamma, prof: int, grid, cut: float,
          bins: Optional[np.ndarray] = None) -> np.ndarray:
    """sigma at all grid points (bins None) or at the given bin indices."""
    nu = _c(nu, np.float64)
    S = _c(S, np.float64)
    alpha = _c(alpha, np.float64)
    gamma = _c(gamma, np.float64)
    if bins is not None:
        bins = _c(bins, np.int64)
        out = np.empty(bins.shape[0])
        nq = bins.shape[0]
    else:
        out = np.empty(grid.n_bins)
        nq = 0
    rc = lib().or_sigma(nu.shape[0], _p(nu), _p(S), _p(alpha), _p(gamma), prof, grid.nu0,
                        grid.dnu, grid.n_bins, cut, nq, _p(bins), _p(out))
    if rc != 0:
        raise MemoryError("oracle sigma: allocation failed")
    return out


def adjoint_sums(nu, alpha, gamma, prof: int, grid, cut: float, g: np.ndarray, absolute: bool = False):
    """Per-line window sums (A, B, C) of g against f, df/dsg and df/dgamma;
    with ``absolute`` the sums of the terms' absolute values."""
    nu = _c(nu, np.float64)
    alpha = _c(alpha, np.float64)
    gamma = _c(gamma, np.float64)
    g = _c(g, np.float64)
    n = nu.shape[0]
    A, B, Cc = np.empty(n), np.empty(n), np.empty(n)
    f = lib().or_adjoint_abs_sums if absolute else lib().or_adjoint_sums
    f(n, _p(nu), _p(alpha), _p(gamma), prof, grid.nu0, grid.dnu, grid.n_bins, cut, _p(g),
      _p(A), _p(B), _p(Cc))
    return A, B, Cc


# ---------------------------------------------------------------------------
# Whole-path helpers
# ---------------------------------------------------------------------------
@dataclass
class CondResult:
    Q: float
    dQdT: float
    nu: np.ndarray
    S: np.ndarray
    keep: np.ndarray
    alpha: np.ndarray
    gamma: np.ndarray
    sigma: Optional[np.ndarray]


def kinetic_T(wl, cond) -> float:
    """Temperature of the line widths: T (LTE) or T_rot (non-LTE)."""
    return cond.T if wl.population == LTE else cond.T_rot


def run_condition(wl, lines, cond, bins: Optional[np.ndarray] = None,
                  log_scale: Optional[np.ndarray] = None, with_sigma: bool = True) -> CondResult:
    """Q -> S_i -> widths -> sigma for one (T, P) or (T_vib, T_rot) condition."""
    Tk = kinetic_T(wl, cond)
    Q, dQ = partition(wl.states, wl.population, cond.T, cond.T_vib, cond.T_rot)
    nu, S, keep = intensities(wl.states, lines, wl.mode, wl.population, cond.T, Q,
                              cond.T_vib, cond.T_rot, log_scale)
    alpha, gamma = widths(nu, lines, wl.profile, Tk, cond.P, wl.mass_amu, wl.T_ref, wl.P_ref,
                          wl.hwhm_fixed, getattr(wl.states, "lifetime", None))
    sig = sigma(nu, S, alpha, gamma, wl.profile, wl.grid, cond.cutoff, bins) if with_sigma else None
    return CondResult(Q, dQ, nu, S, keep, alpha, gamma, sig)


def adjoint(wl, lines, cond, g: np.ndarray, log_scale: Optional[np.ndarray] = None):
    """Gradients of L through sigma for one LTE condition, given g = dL/dsigma.

    sigma_k = sum_i S_i f(nu_k - nu_i; sg_i(T), gamma_i(T, P)), with
    S_i = S_i^0 exp(s_i), sg_i = alpha_i / sqrt(2 ln 2) proportional to sqrt(T),
    gamma_i = gamma_ref,i (T_ref / T)^n_i (P / P_ref).  With per-line window sums
    A_i, B_i, C_i of g against f, df/dsg and df/dgamma:
        dL/ds_i        = S_i A_i
        dL/dgamma_ref,i = S_i C_i gamma_i / gamma_ref,i
        dL/dn_i        = S_i C_i gamma_i ln(T_ref / T)
        dL/dP          = sum_i S_i C_i gamma_i / P
        dL/dT          = sum_i S_i [A_i dlnS_i/dT + B_i sg_i / (2T) - C_i n_i gamma_i / T]
    (the last term of dL/dT is absent for the fixed-HWHM Gaussian, whose width
    does not depend on T; B_i vanishes for the Lorentzian).
    """
    if wl.population != LTE:
        raise ValueError("oracle adjoint: LTE only")
    if wl.profile >= BIN_DOPPLER:
        raise ValueError("oracle adjoint: the sampled Doppler, Gaussian, Lorentzian and Voigt only")
    T, P = cond.T, cond.P
    r = run_condition(wl, lines, cond, log_scale=log_scale, with_sigma=False)
    A, B, Cs = adjoint_sums(r.nu, r.alpha, r.gamma, wl.profile, wl.grid, cond.cutoff, g)
    dlnS = dlnS_dT(wl.states, lines, wl.mode, T, r.Q, r.dQdT)
    sg = r.alpha / np.sqrt(2.0 * np.log(2.0))
    gref = (np.full(lines.n, lines.gamma_ref_scalar) if lines.gamma_ref is None
            else lines.gamma_ref.astype(np.float64))
    nexp = (np.full(lines.n, lines.n_exp_scalar) if lines.n_exp is None
            else lines.n_exp.astype(np.float64))
    S = r.S
    # pressure part of gamma (a lifetime width, if any, depends on none of
    # T, P, gamma_ref, n_exp; the profile sums above use the total width)
    gp = gref * (wl.T_ref / T) ** nexp * (P / wl.P_ref)
    d_s = S * A
    d_gref = S * Cs * (wl.T_ref / T) ** nexp * (P / wl.P_ref)
    d_n = S * Cs * gp * np.log(wl.T_ref / T)
    dsg_dT = sg / (2.0 * T) if wl.profile != GAUSSIAN else np.zeros_like(sg)
    dT_terms = S * (A * dlnS + B * dsg_dT - Cs * nexp * gp / T)
    dP = math.fsum(S * Cs * gp / P) if P > 0 else 0.0
    dT = math.fsum(dT_terms)
    return dict(dT=dT, dP=dP, d_log_scale=d_s, d_gamma_ref=d_gref, d_n_exp=d_n,
                A=A, B=B, C=Cs, S=S, nu=r.nu, alpha=r.alpha, gamma=r.gamma, Q=r.Q, dQdT=r.dQdT)


def adjoint_bounds(wl, lines, cond, g: np.ndarray, log_scale: Optional[np.ndarray] = None):
    """Per-line scales of the adjoint's per-line gradients: each gradient of
    ``adjoint`` with its window sum replaced by the sum of the terms' absolute
    values (``adjoint_sums(..., absolute=True)``) and every factor by its
    absolute value.  |gradient_i| <= bound_i, and a relative error e in every
    term of a window sum moves gradient_i by at most e bound_i: the error of a
    per-line gradient is measured against this scale, since the signed sums
    can cancel to any degree."""
    if wl.population != LTE or wl.profile >= BIN_DOPPLER:
        raise ValueError("oracle adjoint bounds: LTE, sampled profiles only")
    T, P = cond.T, cond.P
    r = run_condition(wl, lines, cond, log_scale=log_scale, with_sigma=False)
    A, _, Cs = adjoint_sums(r.nu, r.alpha, r.gamma, wl.profile, wl.grid, cond.cutoff, g, absolute=True)
    gref = (np.full(lines.n, lines.gamma_ref_scalar) if lines.gamma_ref is None
            else lines.gamma_ref.astype(np.float64))
    nexp = (np.full(lines.n, lines.n_exp_scalar) if lines.n_exp is None
            else lines.n_exp.astype(np.float64))
    S = np.abs(r.S)
    scale = (wl.T_ref / T) ** nexp * (P / wl.P_ref)
    return dict(d_log_scale=S * A, d_gamma_ref=S * Cs * scale,
                d_n_exp=S * Cs * np.abs(gref) * scale * abs(np.log(wl.T_ref / T)))
