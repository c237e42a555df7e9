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

import math

from . import Context, Particles, params_from_preset

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
    """Milliseconds per step of `steps` velocity-Verlet steps on grid ncell ((nx, ny, nz) or n for n^3)."""
    import torch

    params = params_from_preset(preset, prec=prec, ncell=_grid(ncell))
    ctx = Context(params, preset["n"])
    st = Particles.from_numpy(state_np)
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


def batch_params(reps, edge: float, prec: int, xsplit: int = 1):
    """Per-replica params of a batch with cells of edge about `edge` along y and
    z (at least one per axis) and `xsplit` times as many along x."""
    out = []
    for p, _ in reps:
        n = max(1, int(p["L"] // edge))
        out.append(params_from_preset(p, prec=prec, ncell=(xsplit * n, n, n), seed=p["stream_seed"]))
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
