"""GPU parity at the full workload sizes, on sampled particles.

The oracle computes the near field of a sample of particles one by one
(through its cell grid) and the Fourier force of the sample from the
structure factors; the structure factors themselves are checked at sampled
modes. Properties that hold at any size (zero net force, Eq. 12) cover what a
sample cannot.
"""
import importlib.util
import os

import numpy as np
import pytest

import gen
import oracle
from gpu_common import oracle_forces, rel_err, system, to_device

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


def run_full(name, prec, ev=0, nsample=64, nmodes=8):
    p, s = system(name)
    n = p["n"]
    nc = int(p["L"] // EDGE[name])
    params = rbe.params_from_preset(p, prec=prec, ncell=(XSPLIT[name] * nc, nc, nc))
    print(f"{name}: grid {(XSPLIT[name] * nc, nc, nc)}", flush=True)
    ctx = rbe.Context(params, n)
    st = to_device(s)
    m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
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
    P = p["P"]
    rng = np.random.default_rng(7)
    # structure factors at sampled modes
    lm = np.sort(rng.choice(P, size=min(nmodes, P), replace=False))
    re_o, im_o = oracle.rho(s["x"], s["y"], s["z"], s["q"], p["L"], m[:, lm])
    scale = np.sqrt(np.count_nonzero(s["q"]))
    tol_rho = 1e-12 if prec == rbe.FP64 else 1e-6
    assert np.abs(rho[lm] - re_o).max() < tol_rho * scale
    assert np.abs(rho[P + lm] - im_o).max() < tol_rho * scale
    # near field + Fourier force of sampled particles (charged and neutral)
    charged = np.flatnonzero(s["q"] != 0)
    neutral = np.flatnonzero(s["q"] == 0)
    idx = np.concatenate([rng.choice(charged, nsample // 2, replace=False),
                          rng.choice(neutral, nsample // 2, replace=False) if len(neutral) else
                          rng.choice(charged, nsample // 2, replace=False)])
    osys = oracle.sys_from_preset(p)
    FN = oracle.real_force(s["x"], s["y"], s["z"], s["q"], s["id"], osys, seed=p["seed"], ev=ev, idx=idx,
                           cells=True)
    FF, _, _ = oracle.fourier_force(s["x"][idx], s["y"][idx], s["z"][idx], s["q"][idx], p["L"], m, w,
                                    rho[:P], rho[P:])
    return p, s, F, idx, FN, FF


def test_full_electrolyte1m_fp64():
    """1M particles, core-shell list, FP64. Eq. 12's mean is pinned by
    sum_i F_i = 0 (the Fourier part sums to zero) and by the sampled
    differences F_i - F_j, which the mean cancels from."""
    p, s, F, idx, FN, FF = run_full("electrolyte1m", rbe.FP64)
    assert np.abs(F.sum(axis=0)).max() < 1e-9 * np.abs(F).sum() / len(F)
    ref = FN + FF
    mean_est = (ref - F[idx]).mean(axis=0)  # = (1/N) sum_j F~_j, the same for every i
    e = rel_err(F[idx] + mean_est, ref)
    print(f"electrolyte1m FP64 sampled rel err {e:.3e}, mean {mean_est}")
    assert e < 1e-12
    assert np.abs(mean_est).max() < 1.0


def test_full_ljelectrolyte_fp64():
    """The paper's LJ electrolyte at its full size (200,000 ions, L = 271,
    one cutoff r_s = 8, core 4, p = 30), FP64, as for the 1M electrolyte."""
    p, s, F, idx, FN, FF = run_full("ljelectrolyte", rbe.FP64)
    assert np.abs(F.sum(axis=0)).max() < 1e-9 * np.abs(F).sum() / len(F)
    ref = FN + FF
    mean_est = (ref - F[idx]).mean(axis=0)
    e = rel_err(F[idx] + mean_est, ref)
    print(f"ljelectrolyte FP64 sampled rel err {e:.3e}, mean {mean_est}")
    assert e < 1e-12


def test_full_ions8m_fp32c():
    p, s, F, idx, FN, FF = run_full("ions8m", rbe.FP32C)
    e = rel_err(F[idx], FN + FF)
    print(f"ions8m FP32C sampled rel err {e:.3e}")
    assert e < 1e-5
    # FP32 round-off of independent per-particle errors grows like sqrt(N)
    rms = np.sqrt((F ** 2).sum() / len(F))
    assert np.abs(F.sum(axis=0)).max() < 1e-5 * np.sqrt(len(F)) * rms


def test_full_subdomain64m_fp32c():
    p, s, F, idx, FN, FF = run_full("subdomain64m", rbe.FP32C)
    e = rel_err(F[idx], FN + FF)
    print(f"subdomain64m FP32C sampled rel err {e:.3e}")
    assert e < 1e-5


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
