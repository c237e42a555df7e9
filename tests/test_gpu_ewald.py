"""Fixed mode tables on the GPU: with the lattice table of rbe_lattice_modes
the Fourier part is the Ewald reciprocal sum (Eq. 5 over every mode), so
rbe_forces reproduces the oracle's exact Ewald force, and rbe_step with the
table fixed by rbe_set_modes follows the oracle's trajectory under the same
deterministic force."""
import numpy as np
import pytest

from gpu_common import ROW64, max_row_err, rel_err, system, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2609_02694_amd as rbe  # noqa: E402

TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


def kmax_for(alpha, tail=1e-18):
    """|k| beyond which every Ewald coefficient exp(-k^2/4a) is below tail."""
    return float(np.sqrt(4.0 * alpha * np.log(1.0 / tail)))


def oracle_lattice(L, alpha, kmax):
    """The oracle's full lattice (both k and -k) restricted to 0 < |k| <= kmax."""
    M = int(np.floor(kmax * L / (2 * np.pi))) + 1
    m, w = oracle.full_lattice(L, alpha, [M, M, M])
    k2 = ((2 * np.pi / L) ** 2) * (m.astype(np.float64) ** 2).sum(axis=0)
    keep = (k2 > 0) & (k2 <= kmax * kmax)
    return np.ascontiguousarray(m[:, keep]), np.ascontiguousarray(w[keep])


def small_ions(n, L, alpha, r_coul, seed):
    # alpha so large that the screened real-space sum has converged inside
    # r_coul = L/2 (erfc(sqrt(alpha) r_coul) < 1e-16): minimum image suffices
    p, s = system("plain3k", n=n, L=L, alpha=alpha, r_coul=r_coul, seed=seed, density=None)
    return p, s


def device_table(m, w):
    return (torch.as_tensor(np.ascontiguousarray(m, np.int32).ravel()).cuda(),
            torch.as_tensor(np.ascontiguousarray(w, np.float64)).cuda())


def test_lattice_modes_fp32c_match_exact_ewald():
    """FP32C with a full lattice (tens of thousands of modes for a few
    hundred charges: the gather splits the modes over block groups)."""
    L, alpha, rc = 10.0, 1.4, 5.0
    p, s = small_ions(216, L, alpha, rc, seed=2103)
    params = rbe.make_params(L, alpha, rc, 2.5, 1, terms=rbe.TERM_COUL_REAL | rbe.TERM_FOURIER, prec=rbe.FP32C)
    m, w = rbe.lattice_modes(params, kmax_for(alpha))
    params.P = m.shape[1]
    ctx = rbe.Context(params, p["n"])
    st = to_device(s)
    md, wd = device_table(m, w)
    ctx.forces(st, md, wd, 0)
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    torch.cuda.synchronize()
    ctx.sync_check()
    ex = oracle.ewald_exact(s["x"], s["y"], s["z"], s["q"], L, alpha)
    assert rel_err(F, ex["F"]) < 1e-5
    ctx.close()


def test_lattice_modes_give_the_exact_ewald_force():
    L, alpha, rc = 10.0, 1.4, 5.0
    p, s = small_ions(216, L, alpha, rc, seed=2101)
    kmax = kmax_for(alpha)
    params = rbe.make_params(L, alpha, rc, 2.5, 1, terms=rbe.TERM_COUL_REAL | rbe.TERM_FOURIER)
    m, w = rbe.lattice_modes(params, kmax)
    params.P = m.shape[1]
    print(f"exact Ewald: n={p['n']} L={L} alpha={alpha} modes={params.P}", flush=True)
    ctx = rbe.Context(params, p["n"])
    st = to_device(s)
    md, wd = device_table(m, w)
    ctx.forces(st, md, wd, 0)
    F1 = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    ctx.set_modes(md, wd)
    del md, wd  # the context holds its own copy
    ctx.forces(st, None, None, 7)
    F2 = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    torch.cuda.synchronize()
    ctx.sync_check()
    assert np.array_equal(F1, F2)  # explicit table and fixed table: same bits
    ex = oracle.ewald_exact(s["x"], s["y"], s["z"], s["q"], L, alpha)
    assert rel_err(F2, ex["F"]) < TOL64
    assert max_row_err(F2, ex["F"]) < ROW64
    # the Fourier energy of the fixed table is the Ewald reciprocal energy
    u = ctx.energy(st, with_kinetic=False).cpu().numpy()
    assert abs(u[2] - ex["u_recip"]) < 1e-12 * abs(ex["u_recip"])
    assert abs(u[0] - ex["u_real"]) < 1e-12 * abs(ex["u_real"])
    ctx.close()


def test_clearing_the_fixed_table_returns_to_drawing():
    p, s = system("plain3k")
    params = rbe.params_from_preset(p)
    ctx = rbe.Context(params, p["n"])
    st = to_device(s)
    ctx.forces(st, None, None, 3)
    drawn = st.fx.clone()
    m, w = rbe.sample_k(params, 11)
    md, wd = device_table(m, w)
    ctx.set_modes(md, wd)
    ctx.forces(st, None, None, 3)
    assert not torch.equal(st.fx, drawn)  # eval 3 now uses the table of eval 11
    ctx.set_modes(None, None)
    ctx.forces(st, None, None, 3)
    assert torch.equal(st.fx, drawn)
    torch.cuda.synchronize()
    ctx.sync_check()
    ctx.close()


def test_step_with_fixed_lattice_modes_follows_the_oracle():
    """10 NVE steps of Ewald dynamics (lattice table fixed, no batch list):
    positions, velocities and forces match the oracle's velocity Verlet with
    its own full-lattice table."""
    L, alpha, rc = 12.0, 1.0, 6.0
    p, s = small_ions(300, L, alpha, rc, seed=2102)
    n = p["n"]
    kmax = kmax_for(alpha)
    params = rbe.make_params(L, alpha, rc, 2.5, 1, dt=0.002)
    m, w = rbe.lattice_modes(params, kmax)
    params.P = m.shape[1]
    print(f"Ewald dynamics: n={n} modes={params.P}", flush=True)
    ctx = rbe.Context(params, n)
    st = to_device(s)
    md, wd = device_table(m, w)
    ctx.set_modes(md, wd)
    ctx.forces(st, None, None, 0)
    ctx.step(st, 4, 1)
    ctx.step(st, 6, 5)
    torch.cuda.synchronize()
    ctx.sync_check()
    ids = st.id.cpu().numpy()
    mo, wo = oracle_lattice(L, alpha, kmax)
    osys = oracle.make_sys(L, alpha, rc, 2.5)
    r = np.stack([s["x"], s["y"], s["z"]], axis=1)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)

    def force(r):
        return oracle.total_force(r[:, 0], r[:, 1], r[:, 2], s["q"], s["id"], osys, mo, wo)["F"]

    F = force(r)
    for _ in range(10):
        v = oracle.kick(F, v, params.dt / 2)
        r = oracle.drift_wrap(r, v, params.dt, L)
        F = force(r)
        v = oracle.kick(F, v, params.dt / 2)
    gx = np.empty((n, 3)); gv = np.empty((n, 3)); gf = np.empty((n, 3))
    gx[ids] = np.stack([st.x.cpu().numpy(), st.y.cpu().numpy(), st.z.cpu().numpy()], axis=1)
    gv[ids] = np.stack([st.vx.cpu().numpy(), st.vy.cpu().numpy(), st.vz.cpu().numpy()], axis=1)
    gf[ids] = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    d = (gx - r + L / 2) % L - L / 2
    assert np.abs(d).max() < 1e-12 * L
    assert rel_err(gv, v) < TOL64
    assert rel_err(gf, F) < TOL64
    ctx.close()


def test_set_modes_rejected_on_batched_context():
    import gen
    from paper_2609_02694_amd import tune
    reps, cat, off = gen.replica_batch([1000, 1200])
    ctx = rbe.Context.batch(tune.batch_params(reps, 2.5, rbe.FP64, 1), off)
    m, w = rbe.sample_k(ctx.params, 1)
    md, wd = device_table(m, w)
    with pytest.raises(rbe.RbeError) as e:
        ctx.set_modes(md, wd)
    assert "batched" in str(e.value)
    ctx.close()
