"""Autotuner for the cell grid of a system.

The near-field kernels walk, for each particle, the cells of a stencil that
covers its cutoff. Small cells shrink the stencil volume around the cutoff
sphere (fewer candidate pairs) but add cells to walk; the best edge depends
on density, cutoffs and charge fraction. Cells may be split further along x
only: each stencil row is trimmed per particle to the x-cells its cutoff
sphere reaches, so finer x cells cut candidates at the cost of a longer cell
table, without adding rows. tune_grid times a few full steps (binning, near
field, Fourier part, integration) for each candidate (edge, x split) on the
real system and returns the fastest grid.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

from . import TERM_ALL, Context, Particles, params_from_preset

BATCH_EDGES = (2.0, 2.5, 3.0, 3.5, 4.0, 6.0)

DEFAULT_EDGES = (1.25, 1.5, 1.75, 2.0, 2.25, 2.5, 3.0, 3.5, 4.0)

DEFAULT_XSPLITS = (1, 2, 4, 6)


def candidate_grids(L: float, r_max: float, edges=DEFAULT_EDGES, xsplits=(1,)):
    """Grids (nx, n, n) with y/z cell edge about h for h in edges and nx = k n."""
    out = []
    for h in edges:
        n = int(L // h)
        for k in xsplits:
            g = (k * n, n, n)
            if n < 1 or 2 * g[0] * g[1] * g[2] >= (1 << 29) or g in out:
                continue
            out.append(g)
    return out


def _grid(ncell):
    return tuple(ncell) if isinstance(ncell, (tuple, list)) else (ncell, ncell, ncell)


def time_steps(preset: dict, state_np: dict, ncell, prec: int, steps: int = 20, warmup: int = 3) -> float:
    """Milliseconds per step of `steps` steps (velocity Verlet, NVT when the preset asks for it) on grid
    ncell ((nx, ny, nz) or n for n^3)."""
    import torch

    params = params_from_preset(preset, prec=prec, ncell=_grid(ncell))
    ctx = Context(params, preset["n"])
    st = Particles.from_numpy(state_np)
    if preset.get("nvt_tau", 0.0) > 0:
        st.nh = torch.zeros(2, dtype=torch.float64, device="cuda")  # Nose-Hoover {xi, eta}
    ctx.forces(st, None, None, 0)
    ctx.step(st, warmup, 1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.step(st, steps, 1 + warmup)
    e1.record()
    torch.cuda.synchronize()
    ctx.sync_check()
    ctx.close()
    return e0.elapsed_time(e1) / steps


def tune_grid(preset: dict, state_np: dict, prec: int, steps: int = 20, edges=DEFAULT_EDGES,
              xsplits=DEFAULT_XSPLITS, verbose=False):
    """Returns (best (nx, ny, nz), {(nx, ny, nz): ms per step})."""
    r_max = max(preset["r_coul"], preset["r_lj"])
    table = {}
    for g in candidate_grids(preset["L"], r_max, edges, xsplits):
        table[g] = time_steps(preset, state_np, g, prec, steps)
        if verbose:
            print(f"tune: ncell={g} edge={preset['L'] / g[1]:.3f} -> {table[g]:.3f} ms/step", flush=True)
    best = min(table, key=table.get)
    return best, table


def default_ncell(preset: dict) -> int:
    """Grid used without tuning: edge about max(r_lj, r_coul / 3)."""
    h = max(preset["r_lj"] * 0.6, preset["r_coul"] / 3.0)
    return max(1, int(math.floor(preset["L"] / h)))


def batch_params(reps, edge: float, prec: int, xsplit: int = 1, terms: int = TERM_ALL):
    """Per-replica params of a batch with cells of edge about `edge` along y and
    z (at least one per axis) and `xsplit` times as many along x."""
    out = []
    for p, _ in reps:
        n = max(1, int(p["L"] // edge))
        out.append(params_from_preset(p, prec=prec, terms=terms, ncell=(xsplit * n, n, n), seed=p["stream_seed"]))
    return out


def time_batch(reps, cat_np: dict, offsets, edge: float, prec: int, steps: int = 10, warmup: int = 2,
               xsplit: int = 1) -> float:
    """Milliseconds per batched step (all replicas) with cell edge about `edge`."""
    import torch

    ctx = Context.batch(batch_params(reps, edge, prec, xsplit), offsets)
    st = Particles.from_numpy(cat_np)
    ctx.forces(st, None, None, 0)
    ctx.step(st, warmup, 1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.step(st, steps, 1 + warmup)
    e1.record()
    torch.cuda.synchronize()
    ctx.sync_check()
    ctx.close()
    return e0.elapsed_time(e1) / steps


def tune_batch(reps, cat_np: dict, offsets, prec: int, steps: int = 10, edges=BATCH_EDGES, xsplits=(1,),
               verbose=False):
    """Returns (best (edge, xsplit), {(edge, xsplit): ms per step}) for the batched step."""
    table = {}
    for h in edges:
        if min(p["L"] for p, _ in reps) < h:
            continue
        for k in xsplits:
            table[(h, k)] = time_batch(reps, cat_np, offsets, h, prec, steps, xsplit=k)
            if verbose:
                print(f"tune: batch edge {h:.2f} xsplit {k} -> {table[(h, k)]:.3f} ms/step", flush=True)
    best = min(table, key=table.get)
    return best, table


# ---------------------------------------------------------------------------
# cache of tuned grids
# ---------------------------------------------------------------------------
_KEY_FIELDS = ("n", "L", "alpha", "r_coul", "r_lj", "r_core", "p_shell", "P", "ghost", "nvt_tau")


def tune_key(preset: dict, prec: int, kind: str = "grid", extra=None) -> str:
    """Cache key of a tuning problem: the physics and sizes that decide the
    best grid, the precision form, and the GPU it was timed on."""
    dev = "cpu"
    try:
        import torch

        if torch.cuda.is_available():
            dev = torch.cuda.get_device_name(0)
    except Exception:
        pass
    d = {k: preset.get(k) for k in _KEY_FIELDS}
    d.update(kind=kind, prec=int(prec), device=dev, extra=extra)
    return hashlib.sha256(json.dumps(d, sort_keys=True, default=str).encode()).hexdigest()[:24]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, value):
    data = _load(path)
    data[key] = value
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_grid_cached(preset: dict, state_np: dict, prec: int, cache_path: str, steps: int = 20,
                     edges=DEFAULT_EDGES, xsplits=DEFAULT_XSPLITS, verbose=False, timer=None):
    """tune_grid with a JSON cache at cache_path: returns (grid, hit). `timer`
    replaces the step timing (same signature as time_steps), for tests."""
    key = tune_key(preset, prec, "grid", [list(edges), list(xsplits)])
    hit = _load(cache_path).get(key)
    if hit is not None:
        return tuple(hit["grid"]), True
    r_max = max(preset["r_coul"], preset["r_lj"])
    t = timer or time_steps
    table = {g: t(preset, state_np, g, prec, steps) for g in candidate_grids(preset["L"], r_max, edges, xsplits)}
    best = min(table, key=table.get)
    if verbose:
        for g, ms in table.items():
            print(f"tune: ncell={g} -> {ms:.3f} ms/step", flush=True)
    _store(cache_path, key, {"grid": list(best), "ms": {"x".join(map(str, g)): v for g, v in table.items()}})
    return best, False


def tune_batch_cached(reps, cat_np: dict, offsets, prec: int, cache_path: str, steps: int = 10,
                      edges=BATCH_EDGES, xsplits=(1, 2, 3), verbose=False, timer=None):
    """tune_batch with a JSON cache: returns ((edge, xsplit), hit)."""
    sizes = [int(p["n"]) for p, _ in reps]
    key = tune_key(reps[0][0], prec, "batch", [sizes, list(edges), list(xsplits)])
    hit = _load(cache_path).get(key)
    if hit is not None:
        return (hit["edge"], hit["xsplit"]), True
    t = timer or time_batch
    table = {}
    for h in edges:
        if min(p["L"] for p, _ in reps) < h:
            continue
        for k in xsplits:
            table[(h, k)] = t(reps, cat_np, offsets, h, prec, steps, xsplit=k)
            if verbose:
                print(f"tune: batch edge {h:.2f} xsplit {k} -> {table[(h, k)]:.3f} ms/step", flush=True)
    best = min(table, key=table.get)
    _store(cache_path, key, {"edge": best[0], "xsplit": best[1],
                             "ms": {f"{h}/{k}": v for (h, k), v in table.items()}})
    return best, False
