"""Random batch Ewald nonbonded force on one AMD MI355X (gfx950).

Thin binding of the C ABI in ``include/rbe.h`` (library ``libpaper_rbe.so``).
This module only marshals arguments: device memory and streams come from
PyTorch tensors, every step of the computation runs in the HIP kernels. If
the library cannot be loaded the calls raise; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaper_rbe.so")
_lib = None

RBE_OK, RBE_EINVAL, RBE_EBOX, RBE_ENONNEUTRAL, RBE_ENOMEM, RBE_EDEVICE, RBE_ENONFINITE, RBE_ERANGE = (
    0, -1, -2, -3, -4, -5, -6, -7)
FP64, FP32C = 0, 1
KDIST_GAUSS, KDIST_GAUSS_OVER_K2 = 0, 1
SHELL_ALL, SHELL_CHARGED = 0, 1
TERM_LJ, TERM_COUL_REAL, TERM_FOURIER, TERM_ALL = 1, 2, 4, 7
MAX_P = 262144
MAX_SHELL_BATCH = 32

EXPORTED = ["rbe_create", "rbe_create_batch", "rbe_destroy", "rbe_last_error", "rbe_build_cells", "rbe_sample_k",
            "rbe_forces", "rbe_energy", "rbe_step", "rbe_sync_check", "rbe_set_counting", "rbe_get_counters", "rbe_set_timing",
            "rbe_get_timing", "rbe_forces_noalloc", "rbe_lattice_modes", "rbe_set_modes"]
# measurement support (include/rbe_probe.h)
PROBE_EXPORTED = ["rbe_probe_valu"]
PROBE_KINDS = ["fma_f32", "mul_add_f32", "lj_body", "rcp_f32"]
NOALLOC_MAX_N = 32768
NOALLOC_MAX_P = 1024
NOALLOC_MAX_KEYS = 131072
ENERGY_NAMES = ["coul_real", "lj", "fourier", "self", "kinetic", "w_coul_real", "w_lj", "w_fourier"]
TIMING_KINDS = ["bin", "reorder", "pair_neutral", "mean", "sample", "rho_partial", "rho_final", "gather",
                "kick_drift", "kick", "pair_charged", "pair_shell", "ghost", "batch"]


class RbeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rbe status {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_double * 3),
        ("alpha", ctypes.c_double),
        ("r_coul", ctypes.c_double),
        ("r_lj", ctypes.c_double),
        ("r_core", ctypes.c_double),
        ("p_shell", ctypes.c_int32),
        ("P", ctypes.c_int32),
        ("kdist", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("terms", ctypes.c_int32),
        ("ncell", ctypes.c_int32 * 3),
        ("lj_eps", ctypes.c_double),
        ("lj_sigma", ctypes.c_double),
        ("coulomb_k", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("ghost_width", ctypes.c_double),
        ("nvt_kT", ctypes.c_double),
        ("nvt_tau", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("rbl_shell", ctypes.c_int32),
    ]


class State(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "q", "id", "nh")] + [
        ("n", ctypes.c_int64)]


def load():
    """Load the HIP library (built in-tree; built here first if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import _build
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER(Params)
    sig = {
        "rbe_create": [ctypes.POINTER(vp), P, i64, ctypes.c_int],
        "rbe_create_batch": [ctypes.POINTER(vp), i32, P, ctypes.POINTER(i64), ctypes.c_int],
        "rbe_build_cells": [vp, vp, vp, vp, vp, i64, vp, vp, vp],
        "rbe_sample_k": [P, u64, vp, vp, ctypes.c_int, vp],
        "rbe_forces": [vp, ctypes.POINTER(State), vp, vp, u64, vp, vp],
        "rbe_energy": [vp, ctypes.POINTER(State), vp, vp, u64, vp, vp, vp],
        "rbe_step": [vp, ctypes.POINTER(State), i32, u64, vp],
        "rbe_sync_check": [vp, vp],
        "rbe_set_counting": [vp, ctypes.c_int],
        "rbe_get_counters": [vp, ctypes.POINTER(i64), vp],
        "rbe_set_timing": [vp, ctypes.c_int],
        "rbe_get_timing": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), vp],
        "rbe_forces_noalloc": [P, ctypes.POINTER(State), vp, vp, u64, vp, vp, vp],
        "rbe_lattice_modes": [P, ctypes.c_double, vp, vp, i32, ctypes.POINTER(i32)],
        "rbe_set_modes": [vp, vp, vp, vp],
        "rbe_probe_valu": [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_float), vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.rbe_destroy.argtypes = [vp]
    lib.rbe_destroy.restype = None
    lib.rbe_last_error.argtypes = [vp]
    lib.rbe_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def make_params(L, alpha, r_coul, r_lj, P, r_core=0.0, p_shell=0, prec=FP64, terms=TERM_ALL, ncell=(0, 0, 0),
                eps=1.0, sigma=1.0, kc=1.0, mass=1.0, dt=0.002, ghost_width=0.0, seed=0, nvt_kT=0.0,
                nvt_tau=0.0, kdist=KDIST_GAUSS, rbl_shell=SHELL_ALL) -> Params:
    p = Params()
    Lv = L if hasattr(L, "__len__") else (L, L, L)
    for d in range(3):
        p.L[d] = float(Lv[d])
        p.ncell[d] = int(ncell[d])
    p.alpha, p.r_coul, p.r_lj, p.r_core = alpha, r_coul, r_lj, r_core
    p.p_shell, p.P, p.kdist, p.prec, p.terms = p_shell, P, kdist, prec, terms
    p.lj_eps, p.lj_sigma, p.coulomb_k, p.mass, p.dt = eps, sigma, kc, mass, dt
    p.ghost_width, p.seed = ghost_width, seed
    p.nvt_kT, p.nvt_tau = nvt_kT, nvt_tau
    p.rbl_shell = rbl_shell
    return p


def params_from_preset(pr: dict, prec=FP64, terms=TERM_ALL, ncell=(0, 0, 0), seed=None) -> Params:
    return make_params(pr["L"], pr["alpha"], pr["r_coul"], pr["r_lj"], pr["P"], pr.get("r_core", 0.0),
                       pr.get("p_shell", 0), prec, terms, ncell, kc=pr.get("kc", 1.0), dt=pr.get("dt", 0.002),
                       ghost_width=pr.get("ghost", 0.0), seed=pr["seed"] if seed is None else seed,
                       nvt_kT=pr.get("nvt_kT", 0.0), nvt_tau=pr.get("nvt_tau", 0.0),
                       kdist=pr.get("kdist", KDIST_GAUSS), rbl_shell=pr.get("rbl_shell", SHELL_ALL))


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class Particles:
    """Device particle state (torch tensors of one length n)."""
    x: object
    y: object
    z: object
    vx: object
    vy: object
    vz: object
    fx: object
    fy: object
    fz: object
    q: object
    id: object
    nh: object = None  # NVT thermostat state {xi, eta}: float64 CUDA tensor of 2 entries

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def as_struct(self) -> State:
        import torch
        for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "q"):
            t = getattr(self, k)
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.shape[0] != self.n:
                raise ValueError(f"{k} must be a contiguous float64 CUDA tensor of length {self.n}")
        if self.id.dtype != torch.int32 or not self.id.is_cuda or not self.id.is_contiguous():
            raise ValueError("id must be a contiguous int32 CUDA tensor")
        s = State()
        for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "q", "id"):
            setattr(s, k, getattr(self, k).data_ptr())
        if self.nh is not None:
            if self.nh.dtype != torch.float64 or not self.nh.is_cuda or self.nh.numel() < 2:
                raise ValueError("nh must be a float64 CUDA tensor of 2 entries")
            s.nh = self.nh.data_ptr()
        s.n = self.n
        return s

    @staticmethod
    def from_numpy(d: dict, device="cuda"):
        import torch

        def t(a, dt=torch.float64):
            return torch.as_tensor(a, dtype=dt).to(device).contiguous()
        n = len(d["x"])
        z = lambda: torch.zeros(n, dtype=torch.float64, device=device)  # noqa: E731
        return Particles(t(d["x"]), t(d["y"]), t(d["z"]),
                         t(d["vx"]) if "vx" in d else z(), t(d["vy"]) if "vy" in d else z(),
                         t(d["vz"]) if "vz" in d else z(), z(), z(), z(), t(d["q"]), t(d["id"], torch.int32))


def _check(lib, ctx, rc):
    if rc != RBE_OK:
        msg = lib.rbe_last_error(ctx).decode(errors="replace")
        raise RbeError(rc, msg)


def sample_k(params: Params, ev: int, on_device=False, stream=None):
    """Mode sample (m[3, P], w[P]) for evaluation ev (numpy on the host, torch on the device)."""
    lib = load()
    P = params.P
    if on_device:
        import torch
        m = torch.empty(3 * P, dtype=torch.int32, device="cuda")
        w = torch.empty(P, dtype=torch.float64, device="cuda")
        rc = lib.rbe_sample_k(ctypes.byref(params), ev, _ptr(m), _ptr(w), 1, _stream(stream))
        _check(lib, None, rc)
        return m.view(3, P), w
    import numpy as np
    m = np.empty(3 * P, np.int32)
    w = np.empty(P, np.float64)
    rc = lib.rbe_sample_k(ctypes.byref(params), ev, ctypes.c_void_p(m.ctypes.data), ctypes.c_void_p(w.ctypes.data),
                          0, None)
    _check(lib, None, rc)
    return m.reshape(3, P), w


def lattice_modes(params: Params, k_max: float):
    """Ewald reciprocal-sum mode table (m[3, P], w[P], numpy) of the half-space
    lattice modes with 0 < |k| <= k_max (weights doubled for -k)."""
    import numpy as np
    lib = load()
    cnt = ctypes.c_int32()
    _check(lib, None, lib.rbe_lattice_modes(ctypes.byref(params), k_max, None, None, 0, ctypes.byref(cnt)))
    P = cnt.value
    m = np.empty(3 * P, np.int32)
    w = np.empty(P, np.float64)
    _check(lib, None, lib.rbe_lattice_modes(ctypes.byref(params), k_max, ctypes.c_void_p(m.ctypes.data),
                                            ctypes.c_void_p(w.ctypes.data), P, ctypes.byref(cnt)))
    return m.reshape(3, P), w


def probe_valu(kind: str, blocks: int = 4096, iters: int = 4000, stream=None) -> float:
    """Duration in ms of one rbe_probe_valu launch of the given instruction
    mix (PROBE_KINDS; measurement support, see include/rbe_probe.h)."""
    import torch
    lib = load()
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    ms = ctypes.c_float()
    _check(lib, None, lib.rbe_probe_valu(PROBE_KINDS.index(kind), blocks, iters, _ptr(out), ctypes.byref(ms),
                                         _stream(stream)))
    if not torch.isfinite(out).all():
        raise RbeError(RBE_ENONFINITE, f"probe {kind} produced non-finite values")
    return ms.value


def forces_noalloc(params: Params, st: "Particles", m, w, ev: int = 0, rho_out=None, status_out=None,
                   stream=None):
    """rbe_forces without a context or any device allocation (the library's
    file-scope scratch array; see include/rbe.h for the limits). m, w: the
    mode sample (device). status_out: optional device int32 tensor that
    receives the status of the device-side checks."""
    lib = load()
    s = st.as_struct()
    rc = lib.rbe_forces_noalloc(ctypes.byref(params), ctypes.byref(s), _ptr(m), _ptr(w), ev, _ptr(rho_out),
                                _ptr(status_out), _stream(stream))
    _check(lib, None, rc)


class Context:
    """One system on one device (owns the library's scratch)."""

    def __init__(self, params: Params, n_max: int, device: int = 0):
        self.lib = load()
        self.params = params
        h = ctypes.c_void_p()
        rc = self.lib.rbe_create(ctypes.byref(h), ctypes.byref(params), n_max, device)
        _check(self.lib, None, rc)
        self.h = h

    @classmethod
    def batch(cls, params_list, offsets, device: int = 0) -> "Context":
        """Batched context: replica r owns slots [offsets[r], offsets[r + 1]) of every array."""
        self = cls.__new__(cls)
        self.lib = load()
        n_sys = len(params_list)
        if len(offsets) != n_sys + 1:
            raise ValueError("offsets needs n_sys + 1 entries")
        arr = (Params * n_sys)(*params_list)
        off = (ctypes.c_int64 * (n_sys + 1))(*[int(o) for o in offsets])
        self.params = params_list[0]
        self.params_list = list(params_list)
        self.offsets = [int(o) for o in offsets]
        h = ctypes.c_void_p()
        rc = self.lib.rbe_create_batch(ctypes.byref(h), n_sys, arr, off, device)
        _check(self.lib, None, rc)
        self.h = h
        return self

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, rc):
        _check(self.lib, self.h, rc)

    def build_cells(self, x, y, z, q, stream=None):
        import torch
        nkeys = 2 * self.params.ncell[0] * self.params.ncell[1] * self.params.ncell[2]
        if nkeys == 0:
            raise ValueError("build_cells needs an explicit ncell in the params")
        n = int(x.shape[0])
        cs = torch.empty(nkeys + 1, dtype=torch.int32, device=x.device)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
        self._ok(self.lib.rbe_build_cells(self.h, _ptr(x), _ptr(y), _ptr(z), _ptr(q), n, _ptr(cs), _ptr(perm),
                                          _stream(stream)))
        return cs, perm[:n]

    def forces(self, st: Particles, m=None, w=None, ev: int = 0, rho_out=None, stream=None):
        s = st.as_struct()
        self._ok(self.lib.rbe_forces(self.h, ctypes.byref(s), _ptr(m), _ptr(w), ev, _ptr(rho_out),
                                     _stream(stream)))

    def energy(self, st: Particles, m=None, w=None, ev: int = 0, with_kinetic: bool = True, rho_out=None,
               stream=None):
        """Energy and virial terms (device float64 tensor, one entry per ENERGY_NAMES name)."""
        import torch
        s = st.as_struct()
        if not with_kinetic:
            s.vx = s.vy = s.vz = None
        u = torch.empty(len(ENERGY_NAMES), dtype=torch.float64, device=st.x.device)
        self._ok(self.lib.rbe_energy(self.h, ctypes.byref(s), _ptr(m), _ptr(w), ev, _ptr(u), _ptr(rho_out),
                                     _stream(stream)))
        return u

    def step(self, st: Particles, nsteps: int, first_eval: int, stream=None):
        s = st.as_struct()
        self._ok(self.lib.rbe_step(self.h, ctypes.byref(s), nsteps, first_eval, _stream(stream)))

    def set_modes(self, m=None, w=None, stream=None):
        """Fix the mode table (device m[3, P] int32, w[P] float64) for every
        later evaluation with no explicit modes; None returns to drawing."""
        self._ok(self.lib.rbe_set_modes(self.h, _ptr(m), _ptr(w), _stream(stream)))

    def sync_check(self, stream=None):
        self._ok(self.lib.rbe_sync_check(self.h, _stream(stream)))

    def set_counting(self, on: bool):
        self._ok(self.lib.rbe_set_counting(self.h, 1 if on else 0))

    def counters(self, stream=None):
        """Counters of the last evaluation: {part: (coul_pairs, lj_pairs, candidates, shell_members)}."""
        arr = (ctypes.c_int64 * 12)()
        self._ok(self.lib.rbe_get_counters(self.h, arr, _stream(stream)))
        v = list(arr)
        return {name: tuple(v[4 * k: 4 * k + 4]) for k, name in enumerate(("pair_charged", "pair_shell",
                                                                           "pair_neutral"))}

    def set_timing(self, on: bool):
        self._ok(self.lib.rbe_set_timing(self.h, 1 if on else 0))

    def timing(self, stream=None):
        """Per-kernel-kind (summed ms, launch count) since set_timing(True)."""
        ms = (ctypes.c_double * len(TIMING_KINDS))()
        cnt = (ctypes.c_int64 * len(TIMING_KINDS))()
        self._ok(self.lib.rbe_get_timing(self.h, ms, cnt, _stream(stream)))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(TIMING_KINDS)}
