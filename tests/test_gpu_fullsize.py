"""GPU parity at the full workload sizes.

The 1M electrolyte and the paper's 200k LJ electrolyte (random batch list,
Eq. 12) are compared row by row with the oracle's full evaluation. The 8M and
64M systems are compared on about 2,000 sampled rows (charged, neutral, near
a box face, first and last blocks): the oracle computes every structure
factor itself, the near field of each sampled row through its cell grid, and
the Fourier force of the sampled rows from its own structure factors. Each
comparison asserts an RMS bound and a per-row bound.
"""
import importlib.util
import os
import time

import numpy as np
import pytest

import gen
import oracle
from gpu_common import ROW32, ROW64, max_row_err, oracle_forces, rel_err, system, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_02694_amd as rbe  # noqa: E402


def bench_grids():
    """The cell-grid defaults bench.py times (y/z edge, x split per workload)."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py")
    spec = importlib.util.spec_from_file_location("bench_grids", path)
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b.DEFAULT_NCELL_H, b.DEFAULT_XSPLIT


EDGE, XSPLIT = bench_grids()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


def sample_rows(s, nrows, seed=7):
    """Rows compared at full size: charged and neutral particles, particles
    within 0.05 of a box face (they see ghosts or periodic images), and the
    first and last blocks of the particle order."""
    rng = np.random.default_rng(seed)
    n = len(s["x"])
    charged = np.flatnonzero(s["q"] != 0)
    neutral = np.flatnonzero(s["q"] == 0)
    L = float(s["L"][0])
    face = np.flatnonzero((np.minimum(s["x"], L - s["x"]) < 0.05) | (np.minimum(s["y"], L - s["y"]) < 0.05) |
                          (np.minimum(s["z"], L - s["z"]) < 0.05))
    k = nrows // 4
    parts = [rng.choice(charged, min(k, len(charged)), replace=False),
             rng.choice(neutral, min(k, len(neutral)), replace=False) if len(neutral) else
             rng.choice(charged, min(k, len(charged)), replace=False),
             rng.choice(face, min(k, len(face)), replace=False),
             np.arange(n - k // 2, n), np.arange(0, k // 2)]
    return np.unique(np.concatenate(parts).astype(np.int64))


def gpu_full(name, prec, ev, m, w):
    p, s = system(name)
    n = p["n"]
    nc = int(p["L"] // EDGE[name])
    params = rbe.params_from_preset(p, prec=prec, ncell=(XSPLIT[name] * nc, nc, nc))
    print(f"{name}: grid {(XSPLIT[name] * nc, nc, nc)}", flush=True)
    ctx = rbe.Context(params, n)
    st = to_device(s)
    md = torch.as_tensor(m.ravel()).cuda()
    wd = torch.as_tensor(w).cuda()
    rho = torch.zeros(2 * p["P"], dtype=torch.float64, device="cuda")
    ctx.forces(st, md, wd, ev, rho)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    rho = rho.cpu().numpy()
    ctx.close()
    del st
    torch.cuda.empty_cache()
    return p, s, F, rho


def run_full(name, prec, ev=0, nsample=2048):
    """Sampled rows at full size against the oracle: its own structure
    factors (every mode), its near field of each sampled row and its
    Fourier force of the sampled rows."""
    p0 = gen.preset(name)
    m, w = oracle.sample_k(p0["seed"], ev, p0["L"], p0["alpha"], p0["P"])
    p, s, F, rho = gpu_full(name, prec, ev, m, w)
    P = p["P"]
    t0 = time.time()
    re_o, im_o = oracle.rho(s["x"], s["y"], s["z"], s["q"], p["L"], m)
    print(f"{name}: oracle rho ({P} modes) {time.time() - t0:.1f} s", flush=True)
    scale = np.sqrt(np.count_nonzero(s["q"]))
    tol_rho = 1e-12 if prec == rbe.FP64 else 1e-6
    assert np.abs(rho[:P] - re_o).max() < tol_rho * scale
    assert np.abs(rho[P:] - im_o).max() < tol_rho * scale
    idx = sample_rows(s, nsample)
    osys = oracle.sys_from_preset(p)
    t0 = time.time()
    FN = oracle.real_force(s["x"], s["y"], s["z"], s["q"], s["id"], osys, seed=p["seed"], ev=ev, idx=idx,
                           cells=True)
    FF, _, _ = oracle.fourier_force(s["x"][idx], s["y"][idx], s["z"][idx], s["q"][idx], p["L"], m, w, re_o, im_o)
    print(f"{name}: oracle rows ({len(idx)}) {time.time() - t0:.1f} s", flush=True)
    return p, s, F, idx, FN, FF


def run_every_row(name, prec, ev=0):
    """Every row at full size against the oracle's full evaluation, Eq. 12
    mean included (the oracle subtracts its own mean over all N)."""
    p0 = gen.preset(name)
    m, w = oracle.sample_k(p0["seed"], ev, p0["L"], p0["alpha"], p0["P"])
    p, s, F, rho = gpu_full(name, prec, ev, m, w)
    t0 = time.time()
    ref = oracle_forces(p, s, m, w, ev=ev, cells=True)
    print(f"{name}: oracle, every row {time.time() - t0:.1f} s", flush=True)
    return p, s, F, ref


def test_full_electrolyte1m_fp64():
    """1M particles, core-shell list, FP64: every row against the oracle's
    full evaluation, whose Eq. 12 mean is its own (orc_mean_correct over all
    1M near-field forces), so a wrong mean or a wrong unsampled row shows."""
    p, s, F, ref = run_every_row("electrolyte1m", rbe.FP64)
    e, r = rel_err(F, ref["F"]), max_row_err(F, ref["F"])
    print(f"electrolyte1m FP64 every row: rel err {e:.3e}, max row {r:.3e}, oracle mean {ref['mean']}")
    assert e < 1e-12 and r < ROW64
    assert np.abs(F.sum(axis=0)).max() < 1e-9 * np.abs(F).sum() / len(F)


def test_full_ljelectrolyte_fp64():
    """The paper's LJ electrolyte at its full size (200,000 ions, L = 271,
    one cutoff r_s = 8, core 4, p = 30), FP64, every row."""
    p, s, F, ref = run_every_row("ljelectrolyte", rbe.FP64)
    e, r = rel_err(F, ref["F"]), max_row_err(F, ref["F"])
    print(f"ljelectrolyte FP64 every row: rel err {e:.3e}, max row {r:.3e}")
    assert e < 1e-12 and r < ROW64


def test_full_ions8m_fp32c():
    p, s, F, idx, FN, FF = run_full("ions8m", rbe.FP32C)
    ref = FN + FF
    e, r = rel_err(F[idx], ref), max_row_err(F[idx], ref)
    print(f"ions8m FP32C sampled ({len(idx)} rows) rel err {e:.3e}, max row {r:.3e}")
    assert e < 1e-5 and r < ROW32
    # FP32 round-off of independent per-particle errors grows like sqrt(N)
    rms = np.sqrt((F ** 2).sum() / len(F))
    assert np.abs(F.sum(axis=0)).max() < 1e-5 * np.sqrt(len(F)) * rms


@pytest.mark.parametrize("prec", [rbe.FP32C, rbe.FP64])
def test_full_subdomain64m(prec):
    p, s, F, idx, FN, FF = run_full("subdomain64m", prec)
    ref = FN + FF
    e, r = rel_err(F[idx], ref), max_row_err(F[idx], ref)
    print(f"subdomain64m prec={prec} sampled ({len(idx)} rows) rel err {e:.3e}, max row {r:.3e}")
    if prec == rbe.FP64:
        assert e < 1e-12 and r < ROW64
    else:
        assert e < 1e-5 and r < ROW32


def test_full_replica256_batched_fp32c():
    """All 256 replicas (1,000 to 60,000 particles) in one batched context on
    the bench's grids; the smallest, a middle and the largest replica are
    checked whole against the oracle, and every replica's net force is ~0."""
    from paper_2609_02694_amd import tune
    sizes = gen.replica_sizes(256)
    reps, cat, off = gen.replica_batch(sizes)
    print(f"replica256: {int(off[-1])} particles, edge {EDGE['replica']}, x split {XSPLIT['replica']}", flush=True)
    ctx = rbe.Context.batch(tune.batch_params(reps, EDGE["replica"], rbe.FP32C, XSPLIT["replica"]), off)
    st = rbe.Particles.from_numpy(cat)
    ctx.forces(st, None, None, 3)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    ctx.close()
    order = np.argsort(sizes)
    for r in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        p, s = reps[r]
        m, w = oracle.sample_k(p["stream_seed"], 3, p["L"], p["alpha"], p["P"])
        ref = oracle_forces(p, s, m, w, ev=3)["F"]
        e = rel_err(F[off[r]:off[r + 1]], ref)
        print(f"replica {r} (n={p['n']}) rel err {e:.3e}", flush=True)
        assert e < 1e-5
    for r in range(len(reps)):
        Fr = F[off[r]:off[r + 1]]
        rms = np.sqrt((Fr ** 2).sum() / len(Fr))
        assert np.abs(Fr.sum(axis=0)).max() < 1e-5 * np.sqrt(len(Fr)) * rms, r
