"""Seeded synthetic line lists, grids and conditions.

This module only draws random inputs of the shape, size and distribution of the
line-list workloads in the paper's accuracy and performance section (ExoMol-style
states + transitions + broadening, a user wavenumber grid, T/P points).  It holds
none of the method's arithmetic: no intensities, widths, profiles or partition
functions.  The one derived quantity it forms, the transition wavenumber
E_upper - E_lower, is used only to reject pairs outside the requested range.

Both the oracle (tests) and the GPU path (tests, bench) take their inputs from
here.  Every random number comes from NumPy's PCG64 seeded through
``SeedSequence(seed).spawn``: child 0 draws the states, child 1 + j draws line
chunk j, child 1 + n_chunks draws auxiliary vectors (bin weights, cotangents).

Per-line parameters (Einstein A, gamma_ref, n_exp) are rounded to float32 when
drawn, so the FP64 and FP32 forms of the path and the oracle see identical
values.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, List, Optional, Sequence

import numpy as np

# Enumerations mirrored from the C-ABI (include/xsec.h); plain ints here.
DOPPLER, GAUSSIAN, LORENTZ, VOIGT = 0, 1, 2, 3
BIN_DOPPLER, BIN_GAUSSIAN, BIN_LORENTZ, BIN_VOIGT = 4, 5, 6, 7
PV_THOMPSON, PV_OLIVERO = 8, 9
ABSORPTION, EMISSION = 0, 1
LTE, NLTE_2T, NLTE_DENSITY = 0, 1, 2


@dataclass
class States:
    energy: np.ndarray                 # float64 [n], cm^-1
    g_tot: np.ndarray                  # float64 [n]
    v: Optional[np.ndarray] = None     # int32 [n] vibrational manifold (2T only)
    e_vib: Optional[np.ndarray] = None  # float64 [n_v] E_vib(v) (non-LTE only)
    n_vib: Optional[np.ndarray] = None  # float64 [n_v] vibronic densities (custom-density runs)
    lifetime: Optional[np.ndarray] = None  # float64 [n] state lifetimes, s (inf: stable)

    @property
    def n(self) -> int:
        return int(self.energy.shape[0])


@dataclass
class Lines:
    upper: np.ndarray                  # int32 [n]
    lower: np.ndarray                  # int32 [n]
    einstein_a: np.ndarray             # float32 [n], s^-1
    gamma_ref: Optional[np.ndarray] = None  # float32 [n], cm^-1/bar at T_ref, P_ref
    n_exp: Optional[np.ndarray] = None      # float32 [n]
    gamma_ref_scalar: float = 0.07
    n_exp_scalar: float = 0.5

    @property
    def n(self) -> int:
        return int(self.upper.shape[0])

    def take(self, idx: np.ndarray) -> "Lines":
        return Lines(self.upper[idx], self.lower[idx], self.einstein_a[idx],
                     None if self.gamma_ref is None else self.gamma_ref[idx],
                     None if self.n_exp is None else self.n_exp[idx],
                     self.gamma_ref_scalar, self.n_exp_scalar)


@dataclass
class Grid:
    nu0: float
    dnu: float
    n_bins: int


@dataclass
class Condition:
    T: float
    P: float
    cutoff: float
    T_vib: float = 0.0
    T_rot: float = 0.0


@dataclass
class Workload:
    name: str
    states: States
    grid: Grid
    conditions: List[Condition]
    profile: int
    mode: int
    population: int
    mass_amu: float
    n_lines: int
    n_chunks: int
    seed: int
    nu_max: float
    line_kind: str                      # "flat" | "exp" | "manifold"
    hwhm_fixed: float = 0.0
    T_ref: float = 296.0
    P_ref: float = 1.0
    _ss: List[np.random.SeedSequence] = field(default_factory=list, repr=False)
    _lines_cache: Optional[Lines] = field(default=None, repr=False)

    def chunk_sizes(self) -> List[int]:
        base = self.n_lines // self.n_chunks
        sizes = [base] * self.n_chunks
        sizes[-1] += self.n_lines - base * self.n_chunks
        return sizes

    def chunk(self, j: int) -> Lines:
        """Line chunk j, regenerated deterministically from its own seed."""
        rng = np.random.Generator(np.random.PCG64(self._ss[1 + j]))
        return _draw_lines(rng, self.states, self.chunk_sizes()[j], self.nu_max,
                           self.line_kind)

    def chunks(self) -> Iterator[Lines]:
        for j in range(self.n_chunks):
            yield self.chunk(j)

    def lines(self) -> Lines:
        """All lines at once (the 1e9-line workload at full size is streamed chunk by chunk)."""
        if self._lines_cache is None:
            parts = [self.chunk(j) for j in range(self.n_chunks)]
            if len(parts) == 1:
                self._lines_cache = parts[0]
            else:
                self._lines_cache = Lines(
                    np.concatenate([p.upper for p in parts]),
                    np.concatenate([p.lower for p in parts]),
                    np.concatenate([p.einstein_a for p in parts]),
                    None if parts[0].gamma_ref is None else np.concatenate([p.gamma_ref for p in parts]),
                    None if parts[0].n_exp is None else np.concatenate([p.n_exp for p in parts]))
        return self._lines_cache

    def aux_rng(self) -> np.random.Generator:
        return np.random.Generator(np.random.PCG64(self._ss[1 + self.n_chunks]))

    def bin_weights(self) -> np.ndarray:
        """Per-bin loss weights w_k = 10^U(-2, 2) (adjoint workload)."""
        return 10.0 ** self.aux_rng().uniform(-2.0, 2.0, self.grid.n_bins)

    def cotangent(self, n_cond: Optional[int] = None) -> np.ndarray:
        """A seeded dL/dsigma of shape [n_cond, n_bins] with both signs, used to
        drive the adjoint identically on both sides of a parity test."""
        nc = len(self.conditions) if n_cond is None else n_cond
        rng = self.aux_rng()
        rng.uniform(size=self.grid.n_bins)  # skip the weight stream
        return rng.standard_normal((nc, self.grid.n_bins))


def _f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float32)


def _states_flat(rng: np.random.Generator, n: int) -> States:
    E = rng.uniform(0.0, 20000.0, n)
    J = rng.integers(0, 51, n)
    E[0] = 0.0
    J[0] = 0
    return States(E.astype(np.float64), (2 * J + 1).astype(np.float64))


def _states_exp(rng: np.random.Generator, n: int) -> States:
    E = rng.exponential(8000.0, n)
    bad = E > 40000.0
    while bad.any():
        E[bad] = rng.exponential(8000.0, int(bad.sum()))
        bad = E > 40000.0
    J = rng.integers(0, 121, n)
    E[0] = 0.0
    J[0] = 0
    return States(E.astype(np.float64), (2 * J + 1).astype(np.float64))


def _states_manifold(rng: np.random.Generator, n: int) -> States:
    v = rng.integers(0, 11, n)
    J = rng.integers(0, 121, n)
    vv = np.arange(11, dtype=np.float64)
    e_vib = 2000.0 * vv - 10.0 * vv * (vv + 1.0)
    E = e_vib[v] + 1.0 * J * (J + 1.0)
    return States(E.astype(np.float64), (2 * J + 1).astype(np.float64),
                  v.astype(np.int32), e_vib)


def _draw_lines(rng: np.random.Generator, st: States, n: int, nu_max: float,
                kind: str) -> Lines:
    ns = st.n
    E = st.energy
    up = np.empty(0, np.int64)
    lo = np.empty(0, np.int64)
    while up.shape[0] < n:
        m = int((n - up.shape[0]) * 1.25) + 64
        a = rng.integers(0, ns, m)
        b = rng.integers(0, ns, m)
        keep = a != b
        a, b = a[keep], b[keep]
        u = np.where(E[a] > E[b], a, b)
        l = np.where(E[a] > E[b], b, a)
        nu = E[u] - E[l]
        ok = (nu > 0.0) & (nu <= nu_max)
        up = np.concatenate([up, u[ok]])
        lo = np.concatenate([lo, l[ok]])
    up = up[:n].astype(np.int32)
    lo = lo[:n].astype(np.int32)
    if kind == "flat":
        A = _f32(10.0 ** rng.uniform(-6.0, 2.0, n))
        return Lines(up, lo, A)
    A = _f32(10.0 ** rng.uniform(-8.0, 3.0, n))
    if kind == "manifold":
        return Lines(up, lo, A)
    g = _f32(10.0 ** rng.uniform(np.log10(0.02), np.log10(0.1), n))
    ne = _f32(rng.uniform(0.3, 0.8, n))
    return Lines(up, lo, A, g, ne)


GRID48_T = (300.0, 500.0, 800.0, 1200.0, 1800.0, 2500.0, 3500.0, 5000.0)
GRID48_P = (1e-4, 1e-2, 1.0, 10.0, 50.0, 100.0)
TWOTEMP_PAIRS = ((3000.0, 1500.0), (5000.0, 2000.0), (2000.0, 2000.0), (8000.0, 3000.0))

# name -> (seed, states, lines, nu_max, dnu, chunks, line kind, profile, mass)
_WORKLOADS = {
    # LTE absorption, Doppler, 2,000 states, 1e4 lines, grid 0-10000 step 0.01, 1000 K
    "doppler_1e4": (1001, 2000, 10_000, 10000.0, 0.01, 1, "flat", DOPPLER, 18.0),
    # LTE absorption, Voigt, 1e6 states, 1e7 lines, grid 0-20000 step 0.01, 2000 K, 1 bar
    "voigt_1e7": (1002, 1_000_000, 10_000_000, 20000.0, 0.01, 1, "exp", VOIGT, 30.0),
    # the same generator at 1e8 lines under 48 (T, P) conditions
    "voigt_grid48_1e8": (1003, 1_000_000, 100_000_000, 20000.0, 0.01, 1, "exp", VOIGT, 30.0),
    # the 1e7-line Voigt lines driving the adjoint (target spectrum at 1700 K, 0.8 bar)
    "voigt_fit_1e7": (1004, 1_000_000, 10_000_000, 20000.0, 0.01, 1, "exp", VOIGT, 30.0),
    # two-temperature emission, Doppler at T_rot, 1e6 states with v = 0..10,
    # 1e9 lines in 10 chunks, grid 0-30000 step 0.05
    "twotemp_1e9": (1005, 1_000_000, 1_000_000_000, 30000.0, 0.05, 10, "manifold", DOPPLER, 30.0),
}
WORKLOADS = tuple(_WORKLOADS)


def workload(name: str, *, n_lines: Optional[int] = None, n_states: Optional[int] = None,
             nu_hi: Optional[float] = None, n_chunks: Optional[int] = None,
             conditions: Optional[Sequence[Condition]] = None,
             profile: Optional[int] = None, seed: Optional[int] = None) -> Workload:
    """A named workload at full size, or shrunk through the keyword overrides.

    ``nu_hi`` shrinks the line range and the grid together (same step).
    """
    if name not in _WORKLOADS:
        raise ValueError(f"unknown workload {name!r}; one of {WORKLOADS}")
    seed0, ns, nl, hi, dnu, chunks, kind, prof0, mass = _WORKLOADS[name]
    seed = seed0 if seed is None else seed
    if n_states is not None:
        ns = n_states
    if n_lines is not None:
        nl = n_lines
        if n_chunks is None:
            chunks = max(1, min(chunks, nl // 1000))
    if n_chunks is not None:
        chunks = n_chunks
    if nu_hi is not None:
        hi = nu_hi
    n_bins = int(round(hi / dnu)) + 1
    ss = np.random.SeedSequence(seed).spawn(chunks + 2)
    rng = np.random.Generator(np.random.PCG64(ss[0]))
    if kind == "flat":
        st = _states_flat(rng, ns)
    elif kind == "exp":
        st = _states_exp(rng, ns)
    else:
        st = _states_manifold(rng, ns)

    two_temp = name == "twotemp_1e9"
    if conditions is None:
        if name == "doppler_1e4":
            conditions = [Condition(1000.0, 0.0, 25.0)]
        elif name == "voigt_grid48_1e8":
            conditions = [Condition(T, P, 100.0 if P >= 10.0 else 25.0)
                          for T in GRID48_T for P in GRID48_P]
        elif two_temp:
            conditions = [Condition(tr, 0.0, 25.0, T_vib=tv, T_rot=tr) for tv, tr in TWOTEMP_PAIRS]
        else:
            conditions = [Condition(2000.0, 1.0, 25.0)]
    if profile is None:
        profile = prof0
    mode = EMISSION if two_temp else ABSORPTION
    pop = NLTE_2T if two_temp else LTE
    return Workload(name=name, states=st, grid=Grid(0.0, dnu, n_bins),
                    conditions=list(conditions), profile=profile, mode=mode, population=pop,
                    mass_amu=mass, n_lines=nl, n_chunks=chunks, seed=seed, nu_max=hi,
                    line_kind=kind, _ss=ss)


def with_vib_densities(wl: Workload, seed: int = 77) -> Workload:
    """The two-temperature workload's states and lines under user vibronic
    densities instead of T_vib: one weight per manifold, 10^U(-3, 0),
    normalised to sum 1 (the densities' normalisation in the paper's
    custom-density population model).  Only T_rot of each condition is used."""
    if wl.states.e_vib is None:
        raise ValueError("vibronic densities need states with manifolds (the two-temperature workload)")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    w = 10.0 ** rng.uniform(-3.0, 0.0, wl.states.e_vib.shape[0])
    wl.states.n_vib = w / w.sum()
    wl.population = NLTE_DENSITY
    return wl


def with_lifetimes(wl: Workload, frac: float = 0.3, seed: int = 78) -> Workload:
    """Give a fraction of the states finite lifetimes (predissociative states),
    tau = 10^U(-13, -10) s, the rest inf (stable), as an ExoMol states file's
    lifetime column would."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    n = wl.states.n
    tau = np.full(n, np.inf)
    pick = rng.random(n) < frac
    tau[pick] = 10.0 ** rng.uniform(-13.0, -10.0, int(pick.sum()))
    wl.states.lifetime = tau
    return wl


def sample_bins(n_bins: int, n_sample: int, seed: int) -> np.ndarray:
    """Sorted distinct random bin indices for sampled-output parity checks."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    n_sample = min(n_sample, n_bins)
    return np.sort(rng.choice(n_bins, n_sample, replace=False)).astype(np.int64)
