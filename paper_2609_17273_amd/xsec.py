"""Python binding of libxsec (include/xsec.h): argument marshalling only.

Every ``xs_*`` function of the C-ABI has a function of the same name here that
takes ctypes structs / device pointers and returns the status (raising
``XsecError`` on a negative one).  ``Plan`` bundles a plan with a torch-
allocated workspace and takes torch tensors; PyTorch provides device memory
and streams only: every step of the path runs in the library's kernels.
``XsecFunction`` is the autograd wrapper whose backward calls the adjoint.

The library must have been built (``paper_2609_17273_amd.build``); there is no
fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxsec.so")

XS_OK, XS_EINVAL, XS_ENOMEM, XS_EDEVICE, XS_EWORKSPACE, XS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
XS_DOPPLER, XS_GAUSSIAN, XS_LORENTZ, XS_VOIGT = 0, 1, 2, 3
XS_BIN_DOPPLER, XS_BIN_GAUSSIAN, XS_BIN_LORENTZ, XS_BIN_VOIGT = 4, 5, 6, 7
XS_PV_THOMPSON, XS_PV_OLIVERO = 8, 9
XS_ABSORPTION, XS_EMISSION = 0, 1
XS_LTE, XS_NLTE_2T, XS_NLTE_DENSITY = 0, 1, 2
XS_FP64, XS_FP32 = 0, 1
XS_GATHER, XS_SCATTER = 0, 1


class XsecError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"xsec error {code}: {msg}")
        self.code = code


class xs_model(C.Structure):
    _fields_ = [("profile", C.c_int32), ("mode", C.c_int32), ("population", C.c_int32),
                ("precision", C.c_int32), ("algo", C.c_int32), ("mass_amu", C.c_double),
                ("T_ref", C.c_double), ("P_ref", C.c_double), ("hwhm_fixed", C.c_double)]


class xs_grid(C.Structure):
    _fields_ = [("nu0", C.c_double), ("dnu", C.c_double), ("n_bins", C.c_int64)]


class xs_condition(C.Structure):
    _fields_ = [("T", C.c_double), ("P", C.c_double), ("T_vib", C.c_double),
                ("T_rot", C.c_double), ("cutoff", C.c_double)]


class xs_states(C.Structure):
    _fields_ = [("n", C.c_int64), ("energy", C.c_void_p), ("g_tot", C.c_void_p),
                ("v", C.c_void_p), ("e_vib", C.c_void_p), ("n_v", C.c_int32),
                ("n_vib", C.c_void_p), ("lifetime", C.c_void_p)]


class xs_lines(C.Structure):
    _fields_ = [("n", C.c_int64), ("upper", C.c_void_p), ("lower", C.c_void_p),
                ("einstein_a", C.c_void_p), ("gamma_ref", C.c_void_p), ("n_exp", C.c_void_p),
                ("log_scale", C.c_void_p), ("gamma_ref_scalar", C.c_double),
                ("n_exp_scalar", C.c_double)]


class xs_config(C.Structure):
    _fields_ = [("tile_bins", C.c_int32), ("bucket_bins", C.c_int32), ("persistent", C.c_int32),
                ("waves_per_cu", C.c_int32), ("chunk_lines", C.c_int32), ("adj_blocks", C.c_int32)]


class xs_stats(C.Structure):
    _fields_ = [("lines_in", C.c_int64), ("lines_kept", C.c_int64), ("window_pairs", C.c_int64),
                ("work_items", C.c_int64), ("lines_invalid", C.c_int64)]


_P = C.c_void_p
# name -> (restype, argtypes); the exported symbols of include/xsec.h
SIGNATURES = {
    "xs_plan_create": (C.c_int, [C.POINTER(_P), C.POINTER(xs_model), C.POINTER(xs_grid), C.c_int32,
                                 C.POINTER(xs_condition), C.c_int64, _P]),
    "xs_plan_set_conditions": (C.c_int, [_P, C.c_int32, C.POINTER(xs_condition)]),
    "xs_plan_destroy": (None, [_P]),
    "xs_plan_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "xs_plan_set_workspace": (C.c_int, [_P, _P, C.c_size_t]),
    "xs_plan_set_config": (C.c_int, [_P, C.POINTER(xs_config)]),
    "xs_plan_get_config": (C.c_int, [_P, C.POINTER(xs_config)]),
    "xs_partition_function": (C.c_int, [_P, C.POINTER(xs_states), _P, _P]),
    "xs_line_intensities": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), _P, _P]),
    "xs_cross_section": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), _P, C.c_int32]),
    "xs_cross_section_adjoint": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), _P, _P, _P,
                                           _P, _P, _P]),
    "xs_cross_section_noalloc": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), _P, C.c_int32]),
    "xs_prepare": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines)]),
    "xs_profile_pass": (C.c_int, [_P, _P, C.c_int32]),
    "xs_cooling_function": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), C.c_int32, _P, _P, _P]),
    "xs_profile_adjoint": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), _P, _P, _P, _P, _P, _P]),
    "xs_plan_capture": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), _P, C.c_int32]),
    "xs_plan_replay": (C.c_int, [_P]),
    "xs_plan_autotune": (C.c_int, [_P, C.POINTER(xs_states), C.POINTER(xs_lines), _P, C.c_char_p]),
    "xs_plan_get_stats": (C.c_int, [_P, C.POINTER(xs_stats)]),
    "xs_plan_sync": (C.c_int, [_P]),
    "xs_last_error": (C.c_char_p, []),
    "xs_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load libxsec.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2609_17273_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise XsecError(rc, lib().xs_last_error().decode())
    return rc


# ---- the C-ABI, name for name ------------------------------------------------
def xs_plan_create(model, grid, conds, max_lines, stream=None):
    arr = (xs_condition * len(conds))(*conds)
    out = _P()
    _check(lib().xs_plan_create(C.byref(out), C.byref(model), C.byref(grid), len(conds), arr,
                                int(max_lines), stream))
    return out


def xs_plan_set_conditions(plan, conds):
    arr = (xs_condition * len(conds))(*conds)
    return _check(lib().xs_plan_set_conditions(plan, len(conds), arr))


def xs_plan_destroy(plan):
    lib().xs_plan_destroy(plan)


def xs_plan_workspace_bytes(plan) -> int:
    n = C.c_size_t()
    _check(lib().xs_plan_workspace_bytes(plan, C.byref(n)))
    return n.value


def xs_plan_set_workspace(plan, dptr: int, nbytes: int):
    return _check(lib().xs_plan_set_workspace(plan, dptr, nbytes))


def xs_plan_set_config(plan, cfg: xs_config):
    return _check(lib().xs_plan_set_config(plan, C.byref(cfg)))


def xs_plan_get_config(plan) -> xs_config:
    cfg = xs_config()
    _check(lib().xs_plan_get_config(plan, C.byref(cfg)))
    return cfg


def xs_partition_function(plan, states, Q_ptr, dQ_ptr):
    return _check(lib().xs_partition_function(plan, C.byref(states), Q_ptr, dQ_ptr))


def xs_line_intensities(plan, states, lines, S_ptr, log_scale_ptr):
    return _check(lib().xs_line_intensities(plan, C.byref(states), C.byref(lines), S_ptr, log_scale_ptr))


def xs_cross_section(plan, states, lines, sigma_ptr, accumulate=0):
    return _check(lib().xs_cross_section(plan, C.byref(states), C.byref(lines), sigma_ptr, accumulate))


def xs_cross_section_adjoint(plan, states, lines, g_ptr, dT_ptr, dP_ptr, dgref_ptr, dnexp_ptr, dls_ptr):
    return _check(lib().xs_cross_section_adjoint(plan, C.byref(states), C.byref(lines), g_ptr, dT_ptr,
                                                 dP_ptr, dgref_ptr, dnexp_ptr, dls_ptr))


def xs_cross_section_noalloc(plan, states, lines, sigma_ptr, accumulate=0):
    return _check(lib().xs_cross_section_noalloc(plan, C.byref(states), C.byref(lines), sigma_ptr,
                                                 accumulate))


def xs_prepare(plan, states, lines):
    return _check(lib().xs_prepare(plan, C.byref(states), C.byref(lines)))


def xs_profile_pass(plan, sigma_ptr, accumulate=0):
    return _check(lib().xs_profile_pass(plan, sigma_ptr, accumulate))


def xs_cooling_function(plan, states, lines, n_T, T_host_ptr, W_ptr, Q_ptr):
    return _check(lib().xs_cooling_function(plan, C.byref(states), C.byref(lines), n_T, T_host_ptr,
                                            W_ptr, Q_ptr))


def xs_profile_adjoint(plan, states, lines, g_ptr, dT_ptr, dP_ptr, dgref_ptr, dnexp_ptr, dls_ptr):
    return _check(lib().xs_profile_adjoint(plan, C.byref(states), C.byref(lines), g_ptr, dT_ptr, dP_ptr,
                                           dgref_ptr, dnexp_ptr, dls_ptr))


def xs_plan_capture(plan, states, lines, sigma_ptr, accumulate=0):
    return _check(lib().xs_plan_capture(plan, C.byref(states), C.byref(lines), sigma_ptr, accumulate))


def xs_plan_replay(plan):
    return _check(lib().xs_plan_replay(plan))


def xs_plan_autotune(plan, states, lines, sigma_ptr, cache_path: Optional[str] = None):
    return _check(lib().xs_plan_autotune(plan, C.byref(states), C.byref(lines), sigma_ptr,
                                         None if cache_path is None else cache_path.encode()))


def xs_plan_get_stats(plan) -> xs_stats:
    s = xs_stats()
    _check(lib().xs_plan_get_stats(plan, C.byref(s)))
    return s


def xs_plan_sync(plan):
    return _check(lib().xs_plan_sync(plan))


def xs_last_error() -> str:
    return lib().xs_last_error().decode()


def xs_version() -> str:
    return lib().xs_version().decode()


# ---- torch-facing convenience -------------------------------------------------
def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class DeviceStates:
    """States as device tensors (E f64, g f64, optional v i32, e_vib f64,
    n_vib f64 and lifetime f64)."""

    def __init__(self, energy, g_tot, v=None, e_vib=None, n_vib=None, lifetime=None):
        self.energy, self.g_tot, self.v, self.e_vib, self.n_vib = energy, g_tot, v, e_vib, n_vib
        self.lifetime = lifetime

    @classmethod
    def from_numpy(cls, st, device="cuda"):
        import torch
        f = lambda a, dt: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        return cls(f(st.energy, torch.float64), f(st.g_tot, torch.float64), f(st.v, torch.int32),
                   f(st.e_vib, torch.float64), f(getattr(st, "n_vib", None), torch.float64),
                   f(getattr(st, "lifetime", None), torch.float64))

    def struct(self) -> xs_states:
        return xs_states(self.energy.shape[0], _ptr(self.energy), _ptr(self.g_tot), _ptr(self.v),
                         _ptr(self.e_vib), 0 if self.e_vib is None else self.e_vib.shape[0],
                         _ptr(self.n_vib), _ptr(self.lifetime))


class DeviceLines:
    """Transitions as device tensors (upper, lower i32; A, gamma_ref, n_exp, log_scale f32)."""

    def __init__(self, upper, lower, einstein_a, gamma_ref=None, n_exp=None, log_scale=None,
                 gamma_ref_scalar=0.07, n_exp_scalar=0.5):
        self.upper, self.lower, self.einstein_a = upper, lower, einstein_a
        self.gamma_ref, self.n_exp, self.log_scale = gamma_ref, n_exp, log_scale
        self.gamma_ref_scalar, self.n_exp_scalar = gamma_ref_scalar, n_exp_scalar

    @classmethod
    def from_numpy(cls, ln, device="cuda", log_scale=None):
        import torch
        f = lambda a, dt: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        return cls(f(ln.upper, torch.int32), f(ln.lower, torch.int32), f(ln.einstein_a, torch.float32),
                   f(ln.gamma_ref, torch.float32), f(ln.n_exp, torch.float32), f(log_scale, torch.float32),
                   float(ln.gamma_ref_scalar), float(ln.n_exp_scalar))

    @property
    def n(self) -> int:
        return int(self.upper.shape[0])

    def struct(self) -> xs_lines:
        return xs_lines(self.n, _ptr(self.upper), _ptr(self.lower), _ptr(self.einstein_a),
                        _ptr(self.gamma_ref), _ptr(self.n_exp), _ptr(self.log_scale),
                        float(self.gamma_ref_scalar), float(self.n_exp_scalar))


def conditions_of(conds) -> List[xs_condition]:
    return [xs_condition(float(c.T), float(c.P), float(getattr(c, "T_vib", 0.0)),
                         float(getattr(c, "T_rot", 0.0)), float(c.cutoff)) for c in conds]


class Plan:
    """A plan plus its torch-allocated workspace, on torch's current stream."""

    def __init__(self, profile: int, mode: int, population: int, precision: int, grid,
                 conditions, max_lines: int, mass_amu: float = 30.0, algo: int = XS_GATHER,
                 T_ref: float = 296.0, P_ref: float = 1.0, hwhm_fixed: float = 0.0, stream=None):
        import torch
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.model = xs_model(profile, mode, population, precision, algo, mass_amu, T_ref, P_ref, hwhm_fixed)
        self.grid = xs_grid(float(grid.nu0), float(grid.dnu), int(grid.n_bins))
        self.conds = conditions_of(conditions)
        self.n_cond = len(self.conds)
        self.max_lines = int(max_lines)
        self.precision = precision
        self.h = xs_plan_create(self.model, self.grid, self.conds, self.max_lines,
                                _P(stream.cuda_stream))
        self._bind()

    def _bind(self):
        nbytes = xs_plan_workspace_bytes(self.h)
        self.ws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device="cuda")
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        xs_plan_set_workspace(self.h, aligned, nbytes)

    def close(self):
        if getattr(self, "h", None) is not None:
            xs_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_conditions(self, conditions):
        self.conds = conditions_of(conditions)
        try:
            xs_plan_set_conditions(self.h, self.conds)
        except XsecError as e:
            if e.code != XS_EWORKSPACE:
                raise
            self._bind()

    def set_config(self, tile_bins=256, bucket_bins=256, persistent=1, waves_per_cu=16, chunk_lines=0,
                   adj_blocks=0):
        cfg = xs_config(tile_bins, bucket_bins, persistent, waves_per_cu, chunk_lines, adj_blocks)
        try:
            xs_plan_set_config(self.h, cfg)
        except XsecError as e:
            if e.code != XS_EWORKSPACE:
                raise
            self._bind()
            xs_plan_set_config(self.h, cfg)

    def get_config(self) -> dict:
        c = xs_plan_get_config(self.h)
        return dict(tile_bins=c.tile_bins, bucket_bins=c.bucket_bins, persistent=c.persistent,
                    waves_per_cu=c.waves_per_cu, chunk_lines=c.chunk_lines, adj_blocks=c.adj_blocks)

    def partition_function(self, states: DeviceStates):
        t = self.torch
        Q = t.empty(self.n_cond, dtype=t.float64, device="cuda")
        dQ = t.empty(self.n_cond, dtype=t.float64, device="cuda")
        xs_partition_function(self.h, states.struct(), Q.data_ptr(), dQ.data_ptr())
        return Q, dQ

    def line_intensities(self, states: DeviceStates, lines: DeviceLines):
        t = self.torch
        dt = t.float32 if self.precision == XS_FP32 else t.float64
        S = t.empty((self.n_cond, lines.n), dtype=dt, device="cuda")
        ls = t.zeros(self.n_cond, dtype=t.float64, device="cuda")
        xs_line_intensities(self.h, states.struct(), lines.struct(), S.data_ptr(), ls.data_ptr())
        return S, ls

    def cross_section(self, states: DeviceStates, lines: DeviceLines, out=None, accumulate=False):
        t = self.torch
        if out is None:
            out = t.empty((self.n_cond, self.grid.n_bins), dtype=t.float64, device="cuda")
        xs_cross_section(self.h, states.struct(), lines.struct(), out.data_ptr(), int(accumulate))
        return out

    def cross_section_noalloc(self, states: DeviceStates, lines: DeviceLines, out, accumulate=False):
        """xs_cross_section_noalloc into the caller's ``out`` ([n_cond, n_bins]
        float64): the library's static scratch instead of the workspace."""
        xs_cross_section_noalloc(self.h, states.struct(), lines.struct(), out.data_ptr(), int(accumulate))
        return out

    def prepare(self, states: DeviceStates, lines: DeviceLines):
        xs_prepare(self.h, states.struct(), lines.struct())

    def profile(self, out=None, accumulate=False):
        t = self.torch
        if out is None:
            out = t.empty((self.n_cond, self.grid.n_bins), dtype=t.float64, device="cuda")
        xs_profile_pass(self.h, out.data_ptr(), int(accumulate))
        return out

    def profile_adjoint(self, states: DeviceStates, lines: DeviceLines, dL_dsigma):
        return self.adjoint(states, lines, dL_dsigma, prepared=True)

    def cooling_function(self, states: DeviceStates, lines: DeviceLines, T):
        """(W(T), Q(T)) as device tensors for the temperatures T (host sequence)."""
        t = self.torch
        Th = np.ascontiguousarray(np.asarray(T, dtype=np.float64).ravel())
        W = t.empty(Th.shape[0], dtype=t.float64, device="cuda")
        Q = t.empty_like(W)
        xs_cooling_function(self.h, states.struct(), lines.struct(), Th.shape[0],
                            Th.ctypes.data_as(C.c_void_p), W.data_ptr(), Q.data_ptr())
        return W, Q

    def adjoint(self, states: DeviceStates, lines: DeviceLines, dL_dsigma, prepared=False):
        t = self.torch
        g = dL_dsigma.contiguous()
        dT = t.empty(self.n_cond, dtype=t.float64, device="cuda")
        dP = t.empty(self.n_cond, dtype=t.float64, device="cuda")
        dgr = t.empty(lines.n, dtype=t.float64, device="cuda")
        dne = t.empty(lines.n, dtype=t.float64, device="cuda")
        dls = t.empty(lines.n, dtype=t.float64, device="cuda")
        f = xs_profile_adjoint if prepared else xs_cross_section_adjoint
        f(self.h, states.struct(), lines.struct(), g.data_ptr(), dT.data_ptr(), dP.data_ptr(),
          dgr.data_ptr(), dne.data_ptr(), dls.data_ptr())
        return dict(dT=dT, dP=dP, d_gamma_ref=dgr, d_n_exp=dne, d_log_scale=dls)

    def capture(self, states: DeviceStates, lines: DeviceLines, out, accumulate=False):
        xs_plan_capture(self.h, states.struct(), lines.struct(), out.data_ptr(), int(accumulate))

    def replay(self):
        xs_plan_replay(self.h)

    def autotune(self, states: DeviceStates, lines: DeviceLines, scratch, cache_path=None):
        xs_plan_autotune(self.h, states.struct(), lines.struct(), scratch.data_ptr(), cache_path)
        return self.get_config()

    def stats(self) -> dict:
        s = xs_plan_get_stats(self.h)
        return dict(lines_in=s.lines_in, lines_kept=s.lines_kept, window_pairs=s.window_pairs,
                    work_items=s.work_items, lines_invalid=s.lines_invalid)

    def sync(self):
        xs_plan_sync(self.h)


class ChunkStreamer:
    """Line chunks streamed from host memory into one sigma.

    Chunk j+1 is copied from host memory into a pinned staging buffer and then
    to the device on a copy stream, while the plan's stream runs chunk j
    (double buffering); sigma accumulates over the chunks in chunk order, so
    the result equals that of the chunks resident on the device.  Chunks are
    objects with numpy arrays upper, lower (int32), einstein_a, gamma_ref,
    n_exp (float32; gamma_ref / n_exp may be None) and scalars
    gamma_ref_scalar, n_exp_scalar, as produced by the synthetic generator.
    The copies are plumbing: every computation runs in the library's kernels.
    """

    def __init__(self, plan: "Plan", max_chunk_lines: int, copy_threads: int = 8):
        import torch
        from concurrent.futures import ThreadPoolExecutor
        self.torch, self.plan, self.cap = torch, plan, int(max_chunk_lines)
        # host copies into the pinned buffers, split over threads (numpy
        # releases the GIL while copying): one thread copies ~10 GB/s, too
        # slow to keep up with the device on chunks of 1e8 lines
        self.pool = ThreadPoolExecutor(max_workers=max(1, int(copy_threads)))
        n = self.cap
        self.copy_stream = torch.cuda.Stream()  # default priority
        self.host = [self._buffers(n, pinned=True) for _ in range(2)]
        self.dev = [self._buffers(n, pinned=False) for _ in range(2)]
        self.ready = [torch.cuda.Event() for _ in range(2)]      # upload j done
        self.done = [torch.cuda.Event() for _ in range(2)]       # compute on buffer done
        self.copied = [torch.cuda.Event() for _ in range(2)]     # pinned buffer free again

    def _buffers(self, n, pinned):
        t = self.torch
        kw = dict(pin_memory=True) if pinned else dict(device="cuda")
        return dict(upper=t.empty(n, dtype=t.int32, **kw), lower=t.empty(n, dtype=t.int32, **kw),
                    einstein_a=t.empty(n, dtype=t.float32, **kw), gamma_ref=t.empty(n, dtype=t.float32, **kw),
                    n_exp=t.empty(n, dtype=t.float32, **kw))

    def run(self, states: "DeviceStates", chunks, out, accumulate: bool = False):
        """Streams every chunk of the iterable through xs_cross_section into
        out ([n_cond, n_bins] float64); returns the number of lines."""
        t = self.torch
        compute = self.plan.stream
        total = 0
        for j, ch in enumerate(chunks):
            b = j & 1
            n = int(len(ch.upper))
            if n > self.cap:
                raise ValueError(f"chunk of {n} lines exceeds the streamer's {self.cap}")
            h, d = self.host[b], self.dev[b]
            if j >= 2:
                self.copied[b].synchronize()          # the pinned buffer's last upload has left it
            has_g = ch.gamma_ref is not None
            has_n = ch.n_exp is not None
            names = ["upper", "lower", "einstein_a"] + (["gamma_ref"] if has_g else []) + (["n_exp"] if has_n else [])
            self._copy([(h[k][:n].numpy(), getattr(ch, k)) for k in names])
            with t.cuda.stream(self.copy_stream):
                if j >= 2:
                    self.copy_stream.wait_event(self.done[b])  # chunk j-2 no longer reads this buffer
                for k in ("upper", "lower", "einstein_a"):
                    d[k][:n].copy_(h[k][:n], non_blocking=True)
                if has_g:
                    d["gamma_ref"][:n].copy_(h["gamma_ref"][:n], non_blocking=True)
                if has_n:
                    d["n_exp"][:n].copy_(h["n_exp"][:n], non_blocking=True)
                self.copied[b].record(self.copy_stream)
                self.ready[b].record(self.copy_stream)
            compute.wait_event(self.ready[b])
            dl = DeviceLines(d["upper"][:n], d["lower"][:n], d["einstein_a"][:n],
                             d["gamma_ref"][:n] if has_g else None, d["n_exp"][:n] if has_n else None,
                             None, float(ch.gamma_ref_scalar), float(ch.n_exp_scalar))
            with t.cuda.stream(compute):
                self.plan.cross_section(states, dl, out=out, accumulate=accumulate or j > 0)
                self.done[b].record(compute)
            total += n
        compute.synchronize()
        return total

    def _copy(self, pairs, piece: int = 1 << 22):
        jobs = []
        for dst, src in pairs:
            src = np.ascontiguousarray(src, dtype=dst.dtype)
            for a in range(0, dst.shape[0], piece):
                jobs.append(self.pool.submit(np.copyto, dst[a:a + piece], src[a:a + piece]))
        for f in jobs:
            f.result()

    def close(self):
        self.pool.shutdown(wait=True)


def _cond_tuple(conds) -> tuple:
    return tuple((c.T, c.P, c.T_vib, c.T_rot, c.cutoff) for c in conds)


def _make_xsec_function():
    import torch

    class XsecFunction(torch.autograd.Function):
        """sigma(T, P, gamma_ref, n_exp, log_scale) for one plan; backward runs
        the library's adjoint kernel (LTE).  T and P are float64 tensors of
        shape [n_cond]; gamma_ref, n_exp, log_scale float32 tensors [n_lines]
        (the lines' own values, replaced by these)."""

        @staticmethod
        def forward(ctx, T, P, gamma_ref, n_exp, log_scale, plan, states, lines, cutoffs):
            conds = [type("C", (), dict(T=float(t), P=float(p), cutoff=float(c)))()
                     for t, p, c in zip(T.detach().cpu().tolist(), P.detach().cpu().tolist(), cutoffs)]
            plan.set_conditions(conds)
            ln = DeviceLines(lines.upper, lines.lower, lines.einstein_a, gamma_ref.detach().contiguous(),
                             n_exp.detach().contiguous(), log_scale.detach().contiguous())
            sigma = plan.cross_section(states, ln)
            # the conditions of this forward: another apply on the same plan
            # before backward replaces the plan's, and the adjoint must run at
            # these
            ctx.plan, ctx.states, ctx.ln, ctx.conds = plan, states, ln, conds
            return sigma

        @staticmethod
        def backward(ctx, g):
            if _cond_tuple(ctx.plan.conds) != _cond_tuple(conditions_of(ctx.conds)):
                ctx.plan.set_conditions(ctx.conds)
            r = ctx.plan.adjoint(ctx.states, ctx.ln, g.to(torch.float64))
            return (r["dT"], r["dP"], r["d_gamma_ref"].to(torch.float32), r["d_n_exp"].to(torch.float32),
                    r["d_log_scale"].to(torch.float32), None, None, None, None)

    return XsecFunction


_XF = None


def XsecFunction():
    global _XF
    if _XF is None:
        _XF = _make_xsec_function()
    return _XF
