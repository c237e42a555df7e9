"""Autotuner for the cell grid of a system.

The near-field kernels walk, for each particle, the cells of a stencil that
covers its cutoff. Small cells shrink the stencil volume around the cutoff
sphere (fewer candidate pairs) but add cells to walk; the best edge depends
on density, cutoffs and charge fraction. tune_grid times a few full steps
(binning, near field, Fourier part, integration) for each candidate edge on
the real system and returns the fastest grid.
"""
from __future__ import annotations

import math

from . import Context, Particles, params_from_preset

BATCH_EDGES = (2.0, 2.5, 3.0, 3.5, 4.0, 6.0)

DEFAULT_EDGES = (1.25, 1.5, 1.75, 2.0, 2.25, 2.5, 3.0, 3.5, 4.0)


def candidate_grids(L: float, r_max: float, edges=DEFAULT_EDGES):
    out = []
    for h in edges:
        n = int(L // h)
        if n < 1 or (n ** 3) * 2 >= (1 << 29):
            continue
        if n not in out:
            out.append(n)
    return out


def time_steps(preset: dict, state_np: dict, ncell: int, prec: int, steps: int = 20, warmup: int = 3) -> float:
    """Milliseconds per step of `steps` velocity-Verlet steps on grid ncell^3."""
    import torch

    params = params_from_preset(preset, prec=prec, ncell=(ncell, ncell, ncell))
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


def tune_grid(preset: dict, state_np: dict, prec: int, steps: int = 20, edges=DEFAULT_EDGES, verbose=False):
    """Returns (best ncell, {ncell: ms per step})."""
    r_max = max(preset["r_coul"], preset["r_lj"])
    table = {}
    for n in candidate_grids(preset["L"], r_max, edges):
        table[n] = time_steps(preset, state_np, n, prec, steps)
        if verbose:
            print(f"tune: ncell={n} edge={preset['L'] / n:.3f} -> {table[n]:.3f} ms/step", flush=True)
    best = min(table, key=table.get)
    return best, table


def default_ncell(preset: dict) -> int:
    """Grid used without tuning: edge about max(r_lj, r_coul / 3)."""
    h = max(preset["r_lj"] * 0.6, preset["r_coul"] / 3.0)
    return max(1, int(math.floor(preset["L"] / h)))


def batch_params(reps, edge: float, prec: int):
    """Per-replica params of a batch with cells of edge about `edge` (at least one per axis)."""
    out = []
    for p, _ in reps:
        n = max(1, int(p["L"] // edge))
        out.append(params_from_preset(p, prec=prec, ncell=(n, n, n), seed=p["stream_seed"]))
    return out


def time_batch(reps, cat_np: dict, offsets, edge: float, prec: int, steps: int = 10, warmup: int = 2) -> float:
    """Milliseconds per batched step (all replicas) with cell edge about `edge`."""
    import torch

    ctx = Context.batch(batch_params(reps, edge, prec), offsets)
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


def tune_batch(reps, cat_np: dict, offsets, prec: int, steps: int = 10, edges=BATCH_EDGES, verbose=False):
    """Returns (best edge, {edge: ms per step}) for the batched step."""
    table = {}
    for h in edges:
        if min(p["L"] for p, _ in reps) < h:
            continue
        table[h] = time_batch(reps, cat_np, offsets, h, prec, steps)
        if verbose:
            print(f"tune: batch edge {h:.2f} -> {table[h]:.3f} ms/step", flush=True)
    best = min(table, key=table.get)
    return best, table
