"""GPU parity of the batched form: many replicas of uneven size advanced
together (three launches per step), through the C ABI, against the FP64 oracle run
on every replica separately (each replica is its own periodic system with
its own mode sample). FP64 <= 1e-12, FP32C <= 1e-5 (RMS relative, per
replica)."""
import numpy as np
import pytest

import gen
import oracle
from gpu_common import oracle_forces, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_02694_amd as rbe  # noqa: E402

TOL64 = 1e-12
TOL32 = 1e-5

# uneven sizes: the smallest box (L = 12.6, cutoff 6 = L / 2.1) up to 8,000
SMALL = [1000, 2404, 1200, 8000, 1500, 3000]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


def batch_ctx(reps, offsets, prec=rbe.FP64, terms=rbe.TERM_ALL):
    plist = [rbe.params_from_preset(p, prec=prec, terms=terms, seed=p["stream_seed"]) for p, _ in reps]
    return rbe.Context.batch(plist, offsets)


def host(st):
    g = lambda t: t.cpu().numpy()  # noqa: E731
    return dict(x=g(st.x), y=g(st.y), z=g(st.z), vx=g(st.vx), vy=g(st.vy), vz=g(st.vz),
                F=np.stack([g(st.fx), g(st.fy), g(st.fz)], axis=1), q=g(st.q), id=g(st.id))


def replica_oracle(p, s, ev, terms=oracle.LJ | oracle.COUL_REAL | oracle.FOURIER):
    m, w = oracle.sample_k(p["stream_seed"], ev, p["L"], p["alpha"], p["P"])
    return oracle_forces(p, s, m, w, ev=ev, terms=terms)["F"]


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
def test_batched_forces_per_replica(prec, tol):
    reps, cat, off = gen.replica_batch(SMALL)
    print(f"batched forces prec={prec} sizes={SMALL}", flush=True)
    ctx = batch_ctx(reps, off, prec)
    st = rbe.Particles.from_numpy(cat)
    ctx.forces(st, None, None, 7)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = host(st)["F"]
    for r, (p, s) in enumerate(reps):
        ref = replica_oracle(p, s, 7)
        e = rel_err(F[off[r]:off[r + 1]], ref)
        assert e < tol, (r, p["n"], e)
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
def test_batched_forces_split_x_grids(prec, tol):
    """Per-replica grids with x cells finer than y/z cells (per-axis stencil radii)."""
    from paper_2609_02694_amd import tune
    reps, cat, off = gen.replica_batch(SMALL)
    ctx = rbe.Context.batch(tune.batch_params(reps, 2.0, prec, xsplit=3), off)
    st = rbe.Particles.from_numpy(cat)
    ctx.forces(st, None, None, 4)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = host(st)["F"]
    for r, (p, s) in enumerate(reps):
        e = rel_err(F[off[r]:off[r + 1]], replica_oracle(p, s, 4))
        assert e < tol, (r, p["n"], e)
    ctx.close()


@pytest.mark.parametrize("terms", [rbe.TERM_FOURIER, rbe.TERM_COUL_REAL, rbe.TERM_LJ])
def test_batched_terms(terms):
    reps, cat, off = gen.replica_batch(SMALL[:3])
    ctx = batch_ctx(reps, off, rbe.FP64, terms)
    st = rbe.Particles.from_numpy(cat)
    ctx.forces(st, None, None, 3)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = host(st)["F"]
    oterms = {rbe.TERM_FOURIER: oracle.FOURIER, rbe.TERM_COUL_REAL: oracle.COUL_REAL, rbe.TERM_LJ: oracle.LJ}[terms]
    for r, (p, s) in enumerate(reps):
        ref = replica_oracle(p, s, 3, oterms)
        assert rel_err(F[off[r]:off[r + 1]], ref) < TOL64, r
    ctx.close()


def test_batched_equals_single_system_contexts():
    reps, cat, off = gen.replica_batch(SMALL)
    ctx = batch_ctx(reps, off, rbe.FP64)
    st = rbe.Particles.from_numpy(cat)
    ctx.forces(st, None, None, 11)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = host(st)["F"]
    for r, (p, s) in enumerate(reps):
        one = rbe.Context(rbe.params_from_preset(p, seed=p["stream_seed"]), p["n"])
        so = rbe.Particles.from_numpy(s)
        one.forces(so, None, None, 11)
        torch.cuda.synchronize()
        one.sync_check()
        assert rel_err(F[off[r]:off[r + 1]], host(so)["F"]) < TOL64, r
        one.close()
    ctx.close()


def _run_steps(prec, sizes, chunks, first_eval=1):
    """Initial force at eval first_eval - 1, then len(chunks) step calls."""
    reps, cat, off = gen.replica_batch(sizes)
    ctx = batch_ctx(reps, off, prec)
    st = rbe.Particles.from_numpy(cat)
    ctx.forces(st, None, None, first_eval - 1)
    ev = first_eval
    for k in chunks:
        ctx.step(st, k, ev)
        ev += k
    torch.cuda.synchronize()
    ctx.sync_check()
    out = host(st)
    ctx.close()
    return reps, off, out


def _by_id(out, off, r):
    a, b = off[r], off[r + 1]
    ids = out["id"][a:b]
    assert np.array_equal(np.sort(ids), np.arange(b - a))
    res = {}
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        v = np.empty(b - a)
        v[ids] = out[k][a:b]
        res[k] = v
    F = np.empty((b - a, 3))
    F[ids] = out["F"][a:b]
    res["F"] = F
    return res


# FP64: the single-system bounds (1e-12). FP32C: the form's force bound 1e-5;
# per-element force errors of that relative size at the closest LJ contacts
# (|F| up to about 200) move a particle by at most 15 dt^2 x 2e-3 = 1.2e-7 in
# five steps, so positions within 1e-7 L (L >= 12)
@pytest.mark.parametrize("prec,tol_x,tol", [(rbe.FP64, 1e-12, 1e-12), (rbe.FP32C, 1e-7, 1e-5)])
def test_batched_trajectory_against_oracle(prec, tol_x, tol):
    # 5 steps: two graph replays (steps 1-4) and one direct launch (step 5)
    sizes = SMALL[:4]
    reps, off, out = _run_steps(prec, sizes, [5])
    for r, (p, s) in enumerate(reps):
        g = _by_id(out, off, r)
        osys = oracle.sys_from_preset(p)
        rr = np.stack([s["x"], s["y"], s["z"]], axis=1)
        v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)

        def force(rr, ev):
            m, w = oracle.sample_k(p["stream_seed"], ev, p["L"], p["alpha"], p["P"])
            return oracle.total_force(rr[:, 0], rr[:, 1], rr[:, 2], s["q"], s["id"], osys, m, w, ev=ev,
                                      components=False)["F"]
        F = force(rr, 0)
        for k in range(5):
            v = oracle.kick(F, v, p["dt"] / 2)
            rr = oracle.drift_wrap(rr, v, p["dt"], p["L"])
            F = force(rr, k + 1)
            v = oracle.kick(F, v, p["dt"] / 2)
        gx = np.stack([g["x"], g["y"], g["z"]], axis=1)
        d = np.abs(gx - rr)
        d = np.minimum(d, p["L"] - d)  # periodic distance
        gv = np.stack([g["vx"], g["vy"], g["vz"]], axis=1)
        ex, ev_, ef = d.max() / p["L"], rel_err(gv, v), rel_err(g["F"], F)
        print(f"replica {r} (n={p['n']}): |dx|/L {ex:.2e}, v {ev_:.2e}, F {ef:.2e}")
        assert ex < tol_x, r
        assert ev_ < tol, r
        assert ef < tol, r


def test_batched_graph_replays_are_deterministic():
    # 8 steps in one call (four replays of the two-step graph) against
    # 3 + 1 + 4 (direct launches, a fresh chunk layout each call): bit-identical
    sizes = SMALL[:3]
    _, off, a = _run_steps(rbe.FP32C, sizes, [8])
    _, off2, b = _run_steps(rbe.FP32C, sizes, [3, 1, 4])
    for k in ("x", "y", "z", "vx", "vy", "vz", "F", "id"):
        assert np.array_equal(a[k], b[k]), k


def test_batched_rejects_caller_modes_and_charge_imbalance():
    reps, cat, off = gen.replica_batch(SMALL[:2])
    ctx = batch_ctx(reps, off)
    st = rbe.Particles.from_numpy(cat)
    m, w = rbe.sample_k(ctx.params, 0, on_device=True)
    with pytest.raises(rbe.RbeError) as e:
        ctx.forces(st, m.contiguous().view(-1), w, 0)
    assert e.value.code == rbe.RBE_EINVAL
    q = cat["q"].copy()
    i = int(np.nonzero(q[off[1]:] > 0)[0][0]) + off[1]
    q[i] = 0.0  # replica 1 no longer neutral
    st.q.copy_(torch.as_tensor(q))
    ctx.sync_check()
    ctx.forces(st, None, None, 0)  # checked on the device: reported by the next sync_check
    with pytest.raises(rbe.RbeError) as e:
        ctx.sync_check()
    assert e.value.code == rbe.RBE_ENONNEUTRAL and "replica 1" in str(e.value)
    ctx.close()
