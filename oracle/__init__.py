"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle for the RBE nonbonded force.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``rbe_oracle.c`` (plain C,
OpenMP over outer loops) with numpy marshalling and shares no code with the
GPU library.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbe_oracle.c")
_LIB = os.path.join(_HERE, "librbe_oracle.so")
_lib = None

LJ, COUL_REAL, FOURIER = 1, 2, 4
ALL_REAL = LJ | COUL_REAL


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcSys(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("alpha", ctypes.c_double), ("r_coul", ctypes.c_double),
                ("r_lj", ctypes.c_double), ("r_core", ctypes.c_double), ("p_shell", ctypes.c_int32),
                ("eps", ctypes.c_double), ("sigma", ctypes.c_double), ("kc", ctypes.c_double),
                ("shell_charged", ctypes.c_int32)]


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32, i64, u64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    S = ctypes.POINTER(OrcSys)
    sig = {
        "orc_mix64": (u64, [u64]),
        "orc_rbl_key": (ctypes.c_uint32, [u64, u64, i32, i32]),
        "orc_axis_cutoff": (ctypes.c_int, [d, d]),
        "orc_axis_H": (d, [d, d]),
        "orc_norm_S": (d, [_D, d]),
        "orc_norm_S2": (d, [_D, d]),
        "orc_sample_k": (ctypes.c_int, [u64, u64, _D, d, i32, i32, _I32, _D]),
        "orc_rho": (None, [i64, _D, _D, _D, _D, _D, i32, _I32, _D, _D]),
        "orc_fourier_force": (None, [i64, _D, _D, _D, _D, _D, i32, _I32, _D, _D, _D, _D, _D, _D]),
        "orc_fourier_energy": (d, [i32, _D, _D, _D]),
        "orc_real_force": (None, [i64, _D, _D, _D, _D, _I32, S, i32, u64, u64, i64, _I64, _D, _D, _D, _I64]),
        "orc_real_force_cells": (ctypes.c_int, [i64, _D, _D, _D, _D, _I32, S, i32, u64, u64, i64, _I64, _D, _D,
                                                _D]),
        "orc_mean_correct": (None, [i64, _D, _D, _D, _D]),
        "orc_real_energy": (None, [i64, _D, _D, _D, _D, S, _D, _D]),
        "orc_ewald_exact": (None, [i64, _D, _D, _D, _D, _D, d, d, _D, _D, _D, _D, _D, _D]),
        "orc_full_lattice": (i64, [_D, d, _I32, _I32, _D]),
        "orc_self_energy": (d, [i64, _D, d]),
        "orc_fourier_virial": (d, [i32, _I32, _D, d, _D, _D, _D]),
        "orc_real_virial": (None, [i64, _D, _D, _D, _D, S, _D, _D]),
        "orc_kinetic_energy": (d, [i64, _D, _D, _D, d]),
        "orc_bin": (ctypes.c_int, [i64, _D, _D, _D, _D, _D, _I32, _I32, _I32]),
        "orc_kick": (None, [i64, d, _D, _D, _D, _D, _D, _D]),
        "orc_drift_wrap": (None, [i64, d, _D, _D, _D, _D, _D, _D, _D]),
        "orc_num_threads": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(k: int) -> None:
    """Threads of the oracle's parallel loops (the results do not depend on it)."""
    lib = _load()
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads(int(k))


def make_sys(L, alpha, r_coul, r_lj, r_core=0.0, p_shell=0, eps=1.0, sigma=1.0, kc=1.0, shell_charged=0) -> OrcSys:
    s = OrcSys()
    Lv = np.broadcast_to(np.asarray(L, np.float64), (3,))
    for d in range(3):
        s.L[d] = float(Lv[d])
    s.alpha, s.r_coul, s.r_lj, s.r_core = alpha, r_coul, r_lj, r_core
    s.p_shell, s.eps, s.sigma, s.kc = p_shell, eps, sigma, kc
    s.shell_charged = shell_charged
    return s


def sys_from_preset(p: dict) -> OrcSys:
    return make_sys(p["L"], p["alpha"], p["r_coul"], p["r_lj"], p.get("r_core", 0.0), p.get("p_shell", 0),
                    kc=p.get("kc", 1.0), shell_charged=p.get("rbl_shell", 0))


# --------------------------------------------------------------------------
def mix64(z: int) -> int:
    return _load().orc_mix64(z)


def rbl_key(seed, ev, id_i, id_j) -> int:
    return _load().orc_rbl_key(seed, ev, id_i, id_j)


def axis_cutoff(L, alpha) -> int:
    return _load().orc_axis_cutoff(L, alpha)


def axis_H(L, alpha) -> float:
    return _load().orc_axis_H(L, alpha)


def norm_S(L, alpha) -> float:
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    return _load().orc_norm_S(pL, alpha)


def norm_S2(L, alpha) -> float:
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    return _load().orc_norm_S2(pL, alpha)


def sample_k(seed, ev, L, alpha, P, kdist=0):
    """Returns (m[3, P] int32, w[P] float64) of Eq. 9's importance sample."""
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    m = np.empty(3 * P, np.int32)
    w = np.empty(P, np.float64)
    rc = _load().orc_sample_k(seed, ev, pL, alpha, P, kdist, m.ctypes.data_as(_I32), w.ctypes.data_as(_D))
    if rc != 0:
        raise ValueError(f"orc_sample_k status {rc}")
    return m.reshape(3, P), w


def full_lattice(L, alpha, mmax):
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    mm, pm = _i32(np.broadcast_to(np.asarray(mmax, np.int32), (3,)))
    lib = _load()
    cnt = lib.orc_full_lattice(pL, alpha, pm, None, None)
    m = np.empty(3 * cnt, np.int32)
    w = np.empty(cnt, np.float64)
    lib.orc_full_lattice(pL, alpha, pm, m.ctypes.data_as(_I32), w.ctypes.data_as(_D))
    return m.reshape(3, cnt), w


def rho(x, y, z, q, L, m):
    m = np.ascontiguousarray(m, np.int32)
    P = m.shape[1]
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    re = np.empty(P)
    im = np.empty(P)
    _load().orc_rho(len(x), px, py, pz, pq, pL, P, m.ctypes.data_as(_I32), re.ctypes.data_as(_D),
                    im.ctypes.data_as(_D))
    return re, im


def fourier_force(x, y, z, q, L, m, w, rho_re=None, rho_im=None):
    """Eq. 9 estimate for a fixed mode set. Returns (F[n, 3], rho_re, rho_im)."""
    m = np.ascontiguousarray(m, np.int32)
    P = m.shape[1]
    if rho_re is None:
        rho_re, rho_im = rho(x, y, z, q, L, m)
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    (w, pw), (re, pre), (im, pim) = _d(w), _d(rho_re), _d(rho_im)
    n = len(x)
    f = [np.empty(n) for _ in range(3)]
    _load().orc_fourier_force(n, px, py, pz, pq, pL, P, m.ctypes.data_as(_I32), pw, pre, pim,
                              *[a.ctypes.data_as(_D) for a in f])
    return np.stack(f, axis=1), rho_re, rho_im


def fourier_energy(w, rho_re, rho_im) -> float:
    (w, pw), (re, pre), (im, pim) = _d(w), _d(rho_re), _d(rho_im)
    return _load().orc_fourier_energy(len(w), pw, pre, pim)


def real_force(x, y, z, q, ids, sys: OrcSys, terms=ALL_REAL, seed=0, ev=0, idx=None, cells=False,
               return_nshell=False):
    """Near-field force (Eq. 7, 8; Eq. 11 when sys.r_core > 0), before Eq. 12.

    Returns F[len(idx) or n, 3]."""
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    ids, pid = _i32(ids)
    n = len(x)
    if idx is not None:
        idx = np.ascontiguousarray(idx, np.int64)
        cnt = len(idx)
        pidx = idx.ctypes.data_as(_I64)
    else:
        cnt, pidx = n, None
    f = [np.empty(cnt) for _ in range(3)]
    lib = _load()
    if cells:
        rc = lib.orc_real_force_cells(n, px, py, pz, pq, pid, ctypes.byref(sys), terms, seed, ev,
                                      cnt if idx is not None else 0, pidx, *[a.ctypes.data_as(_D) for a in f])
        if rc < 0:
            raise MemoryError("orc_real_force_cells")
        nsh = None
    else:
        nsh = np.empty(cnt, np.int64)
        lib.orc_real_force(n, px, py, pz, pq, pid, ctypes.byref(sys), terms, seed, ev,
                           cnt if idx is not None else 0, pidx, *[a.ctypes.data_as(_D) for a in f],
                           nsh.ctypes.data_as(_I64))
    F = np.stack(f, axis=1)
    return (F, nsh) if return_nshell else F


def mean_correct(F):
    F = np.array(F, dtype=np.float64, order="C")
    cols = [np.ascontiguousarray(F[:, d]) for d in range(3)]
    mean = np.empty(3)
    _load().orc_mean_correct(F.shape[0], *[c.ctypes.data_as(_D) for c in cols], mean.ctypes.data_as(_D))
    return np.stack(cols, axis=1), mean


def real_energy(x, y, z, q, sys: OrcSys):
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    uc, ul = ctypes.c_double(), ctypes.c_double()
    _load().orc_real_energy(len(x), px, py, pz, pq, ctypes.byref(sys), ctypes.byref(uc), ctypes.byref(ul))
    return uc.value, ul.value


def fourier_virial(m, L, alpha, w, rho_re, rho_im) -> float:
    m = np.ascontiguousarray(m, np.int32)
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    (w, pw), (re, pre), (im, pim) = _d(w), _d(rho_re), _d(rho_im)
    return _load().orc_fourier_virial(len(w), m.ctypes.data_as(_I32), pL, alpha, pw, pre, pim)


def real_virial(x, y, z, q, sys: OrcSys):
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    wc, wl = ctypes.c_double(), ctypes.c_double()
    _load().orc_real_virial(len(x), px, py, pz, pq, ctypes.byref(sys), ctypes.byref(wc), ctypes.byref(wl))
    return wc.value, wl.value


def self_energy(q, alpha) -> float:
    (q, pq) = _d(q)
    return _load().orc_self_energy(len(q), pq, alpha)


def kinetic_energy(v, mass) -> float:
    v = np.asarray(v, np.float64)
    cols = [_d(v[:, d]) for d in range(3)]
    return _load().orc_kinetic_energy(v.shape[0], *[c[1] for c in cols], mass)


def ewald_exact(x, y, z, q, L, alpha, tol=1e-17):
    """Exact Ewald energy parts (real, recip, self) and total force."""
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    n = len(x)
    ur, uk, us = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    f = [np.empty(n) for _ in range(3)]
    _load().orc_ewald_exact(n, px, py, pz, pq, pL, alpha, tol, ctypes.byref(ur), ctypes.byref(uk), ctypes.byref(us),
                            *[a.ctypes.data_as(_D) for a in f])
    return dict(u_real=ur.value, u_recip=uk.value, u_self=us.value,
                u=ur.value + uk.value - us.value, F=np.stack(f, axis=1))


def bin_cells(x, y, z, q, L, ncell):
    """Stable counting sort by (species, cell). Returns (cell_start[2*ncell+1], perm[n])."""
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    nc, pnc = _i32(np.broadcast_to(np.asarray(ncell, np.int32), (3,)))
    nkeys = 2 * int(nc[0]) * int(nc[1]) * int(nc[2])
    cs = np.empty(nkeys + 1, np.int32)
    perm = np.empty(len(x), np.int32)
    rc = _load().orc_bin(len(x), px, py, pz, pq, pL, pnc, cs.ctypes.data_as(_I32), perm.ctypes.data_as(_I32))
    if rc != 0:
        raise MemoryError("orc_bin")
    return cs, perm


def kick(F, v, half_dt_over_m):
    v = np.array(v, dtype=np.float64, order="C")
    cols = [np.ascontiguousarray(v[:, d]) for d in range(3)]
    F = np.asarray(F, np.float64)
    fc = [np.ascontiguousarray(F[:, d]) for d in range(3)]
    _load().orc_kick(len(cols[0]), half_dt_over_m, *[c.ctypes.data_as(_D) for c in fc],
                     *[c.ctypes.data_as(_D) for c in cols])
    return np.stack(cols, axis=1)


def drift_wrap(r, v, dt, L):
    r = np.asarray(r, np.float64)
    v = np.asarray(v, np.float64)
    rc = [np.ascontiguousarray(r[:, d]) for d in range(3)]
    vc = [np.ascontiguousarray(v[:, d]) for d in range(3)]
    Lv, pL = _d(np.broadcast_to(np.asarray(L, np.float64), (3,)))
    _load().orc_drift_wrap(len(rc[0]), dt, pL, *[c.ctypes.data_as(_D) for c in vc], *[c.ctypes.data_as(_D) for c in rc])
    return np.stack(rc, axis=1)


# --------------------------------------------------------------------------
# Composite evaluations used by the tests and the CPU baseline
# --------------------------------------------------------------------------
def total_force(x, y, z, q, ids, sys: OrcSys, m, w, seed=0, ev=0, terms=LJ | COUL_REAL | FOURIER, cells=None,
                components=True):
    """F = F^N (Eq. 7 near field, with Eq. 11-12 when the list is on) + F^F (Eq. 9).

    Returns dict with the total and (components=True) each near-field term."""
    n = len(x)
    if cells is None:
        cells = n > 20000
    out = {}
    FN = np.zeros((n, 3))
    if components and terms & LJ:
        out["lj"] = real_force(x, y, z, q, ids, sys, LJ, seed, ev, cells=cells)
    if components and terms & COUL_REAL:
        out["coul"] = real_force(x, y, z, q, ids, sys, COUL_REAL, seed, ev, cells=cells)
    if terms & (LJ | COUL_REAL):
        FN = real_force(x, y, z, q, ids, sys, terms & (LJ | COUL_REAL), seed, ev, cells=cells)
        if sys.r_core > 0 and sys.p_shell > 0:
            FN, mean = mean_correct(FN)
            out["mean"] = mean
    FF = np.zeros((n, 3))
    if terms & FOURIER:
        FF, re, im = fourier_force(x, y, z, q, sys.L, m, w)
        FF = sys.kc * FF  # the Coulomb prefactor scales the Fourier part too
        out["rho_re"], out["rho_im"] = re, im
    out["fourier"] = FF
    out["near"] = FN
    out["F"] = FN + FF
    return out


def nh_half(K, xi, eta, dt, nf, kT, Q):
    """One half-step of a single Nose-Hoover thermostat (Hoover 1985, the
    thermostat of the paper's NVT runs), symmetric Trotter split:
    xi += dt/4 G(K); s = exp(-xi dt/2); eta += xi dt/2; K <- s^2 K;
    xi += dt/4 G(K), with G(K) = (2K - nf kT)/Q. Returns (s, K, xi, eta);
    the velocities are to be multiplied by s."""
    xi = xi + 0.25 * dt * ((2.0 * K - nf * kT) / Q)
    s = math.exp(-0.5 * dt * xi)
    eta = eta + 0.5 * dt * xi
    K = K * s * s
    xi = xi + 0.25 * dt * ((2.0 * K - nf * kT) / Q)
    return s, K, xi, eta


def nvt_step(r, v, F, xi, eta, force, dt, L, mass, kT, tau):
    """One NVT step: thermostat half, velocity-Verlet step with force(r),
    thermostat half. Q = nf kT tau^2 with nf = 3N - 3. Returns (r, v, F, xi, eta)."""
    nf = 3.0 * len(r) - 3.0
    Q = nf * kT * tau * tau
    s, _, xi, eta = nh_half(kinetic_energy(v, mass), xi, eta, dt, nf, kT, Q)
    v = v * s
    v = kick(F, v, 0.5 * dt / mass)
    r = drift_wrap(r, v, dt, L)
    F = force(r)
    v = kick(F, v, 0.5 * dt / mass)
    s, _, xi, eta = nh_half(kinetic_energy(v, mass), xi, eta, dt, nf, kT, Q)
    return r, v * s, F, xi, eta


def energy_terms(x, y, z, q, sys: OrcSys, m, w, v=None, mass=1.0, terms=LJ | COUL_REAL | FOURIER):
    """Energy and virial terms of Sec. 2.1 for a fixed mode sample (m, w):
    coul_real = kc sum_{i<j} q_i q_j erfc(sqrt(a) r)/r within r_coul (Eq. 4),
    lj = sum_{i<j} 4 eps ((sigma/r)^12 - (sigma/r)^6) within r_lj (Eq. 2),
    fourier = kc (1/2) sum_l w_l |rho_l|^2 (Eq. 5 sampled as in Eq. 9),
    self = kc sqrt(a/pi) sum q^2 (Eq. 6), kinetic = (m/2) sum |v|^2, and the
    virials w_coul_real, w_lj (sum_{i<j} d_ij . F_ij) and w_fourier
    (kc (1/2) sum_l w_l |rho_l|^2 (1 - k_l^2/(2a))). The potential is
    coul_real + lj + fourier - self; its negative gradient at fixed modes is
    total_force without the random batch list; the pressure is
    (2 kinetic + w_coul_real + w_lj + w_fourier) / (3 V)."""
    uc, ul = real_energy(x, y, z, q, sys)
    wc, wl = real_virial(x, y, z, q, sys)
    out = dict(coul_real=uc if terms & COUL_REAL else 0.0, lj=ul if terms & LJ else 0.0, fourier=0.0, self=0.0)
    if terms & FOURIER:
        re, im = rho(x, y, z, q, sys.L, m)
        out["fourier"] = sys.kc * fourier_energy(w, re, im)
        out["self"] = sys.kc * self_energy(q, sys.alpha)
    out["kinetic"] = kinetic_energy(v, mass) if v is not None else 0.0
    out["w_coul_real"] = wc if terms & COUL_REAL else 0.0
    out["w_lj"] = wl if terms & LJ else 0.0
    out["w_fourier"] = sys.kc * fourier_virial(m, sys.L, sys.alpha, w, re, im) if terms & FOURIER else 0.0
    out["potential"] = out["coul_real"] + out["lj"] + out["fourier"] - out["self"]
    return out
