"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Nothing here computes any part of the random batch Ewald method: the module
draws positions (random sequential addition with a minimum separation),
charges (exact +/- counts, shuffled) and Maxwell-Boltzmann velocities, and
holds the workload presets. See ``rbe_gen.c`` for the generator definitions.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbe_gen.c")
_LIB = os.path.join(_HERE, "librbe_gen.so")
_lib = None


def build() -> str:
    """Compile the generator with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", _SRC, "-o", _LIB + ".tmp",
           "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    d, i64, u64 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64
    dp = ctypes.POINTER(ctypes.c_double)
    lib.gen_rsa_positions.argtypes = [u64, u64, i64, dp, d, i64, dp, dp, dp]
    lib.gen_rsa_blocked.argtypes = [u64, u64, i64, dp, d, d, i64, dp, dp, dp]
    lib.gen_charges.argtypes = [u64, u64, i64, i64, i64, d, dp]
    lib.gen_velocities.argtypes = [u64, u64, i64, d, d, dp, dp, dp]
    for f in (lib.gen_rsa_positions, lib.gen_rsa_blocked, lib.gen_charges, lib.gen_velocities):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def rsa_positions(seed: int, replica: int, n: int, L, dmin: float = 0.8, max_attempts: int = 100000):
    lib = _load()
    Lv = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    x, y, z = (np.empty(n, np.float64) for _ in range(3))
    rc = lib.gen_rsa_positions(seed, replica, n, _ptr(Lv), dmin, max_attempts, _ptr(x), _ptr(y), _ptr(z))
    if rc != 0:
        raise RuntimeError(f"gen_rsa_positions failed with status {rc}")
    return x, y, z


def rsa_blocked(seed: int, replica: int, n: int, L, dmin: float = 0.8, block_edge: float = 4.0,
                max_attempts: int = 100000):
    """Blocked RSA (parallel, deterministic): see gen_rsa_blocked in rbe_gen.c."""
    lib = _load()
    Lv = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    x, y, z = (np.empty(n, np.float64) for _ in range(3))
    rc = lib.gen_rsa_blocked(seed, replica, n, _ptr(Lv), dmin, block_edge, max_attempts, _ptr(x), _ptr(y), _ptr(z))
    if rc != 0:
        raise RuntimeError(f"gen_rsa_blocked failed with status {rc}")
    return x, y, z


# systems at or above this size use the blocked RSA
BLOCKED_RSA_MIN_N = 2_000_000


def charges(seed: int, replica: int, n: int, n_plus: int, n_minus: int, qmag: float = 1.0):
    lib = _load()
    q = np.empty(n, np.float64)
    rc = lib.gen_charges(seed, replica, n, n_plus, n_minus, qmag, _ptr(q))
    if rc != 0:
        raise RuntimeError(f"gen_charges failed with status {rc}")
    return q


def velocities(seed: int, replica: int, n: int, kT: float = 1.0, mass: float = 1.0):
    lib = _load()
    vx, vy, vz = (np.empty(n, np.float64) for _ in range(3))
    rc = lib.gen_velocities(seed, replica, n, kT, mass, _ptr(vx), _ptr(vy), _ptr(vz))
    if rc != 0:
        raise RuntimeError(f"gen_velocities failed with status {rc}")
    return vx, vy, vz


# ---------------------------------------------------------------------------
# Workload presets: charged Lennard-Jones systems in a cubic periodic box.
# Every preset uses eps = sigma = 1, mass 1, kT = 1, Coulomb prefactor 1.
# ---------------------------------------------------------------------------

PRESETS = {
    # N = 3,000 point charges (half +1, half -1), L = 30, cutoff 8, P = 100.
    "plain3k": dict(seed=1001, n=3000, density=None, L=30.0, frac_charged=1.0, alpha=0.3,
                    r_coul=8.0, r_lj=2.5, r_core=0.0, p_shell=0, P=100, dt=0.002, ghost=0.0),
    # N = 1,000,000 at number density 0.8, 25 % ions, core-shell list (core 3, batch 20), P = 200.
    "electrolyte1m": dict(seed=1002, n=1_000_000, density=0.8, L=None, frac_charged=0.25, alpha=0.35,
                          r_coul=6.0, r_lj=2.5, r_core=3.0, p_shell=20, P=200, dt=0.002, ghost=0.0),
    # N = 8,000,000 all ions at the density of the 3k case, cutoff 8, P = 500.
    "ions8m": dict(seed=1003, n=8_000_000, density=3000 / 30.0 ** 3, L=None, frac_charged=1.0, alpha=0.3,
                   r_coul=8.0, r_lj=2.5, r_core=0.0, p_shell=0, P=500, dt=0.002, ghost=0.0),
    # One replica shape of the 256-replica batch (N set per replica), density 0.5, half ions.
    "replica": dict(seed=1004, n=None, density=0.5, L=None, frac_charged=0.5, alpha=0.3,
                    r_coul=6.0, r_lj=2.5, r_core=0.0, p_shell=0, P=100, dt=0.002, ghost=0.0),
    # N = 64,000,000 at density 0.8, 10 % ions, 6-sigma ghost shell built locally, P = 1000.
    "subdomain64m": dict(seed=1005, n=64_000_000, density=0.8, L=None, frac_charged=0.10, alpha=0.35,
                         r_coul=6.0, r_lj=2.5, r_core=0.0, p_shell=0, P=1000, dt=0.002, ghost=6.0),
    # The paper's implicit-solvent LJ electrolyte (Sec. 3.1 and its parameter table): N = 200,000
    # monovalent ions, L = 271, one short-range cutoff r_s = 8 for LJ and Coulomb, core r_c = 4,
    # batch p = 30, P = 200, dt = 0.001, Nose-Hoover at kT = 1 (relaxation time 100 dt). alpha is
    # not printed: sqrt(alpha) r_s = 3 (erfc(3) = 2.2e-5, below the 1e-4 the paper asks of PPPM).
    "ljelectrolyte": dict(seed=1006, n=200_000, density=200_000 / 271.0 ** 3, L=271.0, frac_charged=1.0,
                              alpha=(3.0 / 8.0) ** 2, r_coul=8.0, r_lj=8.0, r_core=4.0, p_shell=30, P=200,
                              dt=0.001, ghost=0.0, nvt_kT=1.0, nvt_tau=0.1),
}


def replica_sizes(count: int = 256, seed: int = 1004, lo: int = 1000, hi: int = 60000):
    """Log-uniform replica sizes in [lo, hi], rounded to a multiple of 4."""
    # SplitMix64 stream, as in rbe_gen.c
    g = 0x9E3779B97F4A7C15
    mask = (1 << 64) - 1

    def mix64(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        return z ^ (z >> 31)

    key = mix64(((seed ^ 0x5245504C49434153) + g) & mask)  # tag "REPLICAS"
    out = []
    for r in range(count):
        u = (mix64((key + (r + 1) * g) & mask) >> 11) * 2.0 ** -53
        n = math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
        n = int(round(n / 4.0)) * 4
        out.append(min(max(n, lo), hi))
    return out


def preset(name: str, n: int | None = None, **overrides) -> dict:
    """Return the preset with N (and the box at the preset density) resolved."""
    p = dict(PRESETS[name])
    p.update(overrides)
    if n is not None:
        p["n"] = int(n)
    if p["n"] is None:
        raise ValueError("preset needs n")
    if p.get("density") is not None and (p.get("L") is None or n is not None):
        p["L"] = (p["n"] / p["density"]) ** (1.0 / 3.0)
    p["name"] = name
    return p


def make_system(p: dict, replica: int = 0, dmin: float = 0.8) -> dict:
    """Draw positions, charges, velocities and ids for preset ``p``.

    Charges: round(N * frac_charged / 2) at +1 and the same number at -1, so
    the system is exactly neutral.
    """
    n = p["n"]
    L = p["L"]
    seed = p["seed"]
    if n >= BLOCKED_RSA_MIN_N:
        x, y, z = rsa_blocked(seed, replica, n, [L, L, L], dmin)
    else:
        x, y, z = rsa_positions(seed, replica, n, [L, L, L], dmin)
    nq = int(round(n * p["frac_charged"] / 2.0))
    q = charges(seed, replica, n, nq, nq)
    vx, vy, vz = velocities(seed, replica, n)
    ids = np.arange(n, dtype=np.int32)
    return dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, q=q, id=ids, L=np.array([L, L, L], np.float64))


def replica_stream_seed(seed: int, replica: int) -> int:
    """Stream seed of replica ``replica``'s mode sample (distinct per replica)."""
    return ((seed << 16) + replica) & ((1 << 64) - 1)


def replica_batch(sizes, name: str = "replica"):
    """Presets and systems of a batch of replicas of the given sizes.

    Replica r draws its particles as replica r of the preset's seed; its
    mode-sample stream seed is ``replica_stream_seed(seed, r)`` (stored as
    ``p["stream_seed"]``). Returns the list of (preset, system) pairs, the
    concatenated system (ids local to each replica) and the offsets."""
    reps = []
    for r, n in enumerate(sizes):
        p = preset(name, n=int(n))
        p["stream_seed"] = replica_stream_seed(p["seed"], r)
        reps.append((p, make_system(p, replica=r)))
    keys = ("x", "y", "z", "vx", "vy", "vz", "q", "id")
    cat = {k: np.concatenate([s[k] for _, s in reps]) for k in keys}
    offsets = np.concatenate([[0], np.cumsum([len(s["x"]) for _, s in reps])]).astype(np.int64)
    return reps, cat, offsets
