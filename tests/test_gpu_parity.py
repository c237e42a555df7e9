"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

FP64 path: RMS relative force error <= 1e-12 (per term and total).
FP32C path: <= 1e-5. Integer work (binning, mode sample, batch selection):
bit-exact.
"""
import numpy as np
import pytest

import gen
import oracle
from gpu_common import ROW32, ROW64, gpu_forces, max_row_err, oracle_forces, rel_err, system, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_02694_amd as rbe  # noqa: E402

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


# ---------------------------------------------------------------------------
# mode sampler
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,alpha,P", [(30.0, 0.3, 100), (107.72, 0.35, 200), (416.02, 0.3, 500), (12.6, 0.3, 7)])
def test_sample_k_device_equals_host_and_oracle(L, alpha, P):
    p = rbe.make_params(L, alpha, 2.0, 1.0, P, seed=1234)
    for ev in (0, 1, 977):
        mh, wh = rbe.sample_k(p, ev)
        md, wd = rbe.sample_k(p, ev, on_device=True)
        assert np.array_equal(mh, md.cpu().numpy()) and np.array_equal(wh, wd.cpu().numpy())
        mo, wo = oracle.sample_k(1234, ev, L, alpha, P)
        assert np.array_equal(mh, mo) and np.array_equal(wh, wo)


@pytest.mark.parametrize("L,alpha,P", [(30.0, 0.3, 100), (107.72, 0.35, 50), (12.6, 0.3, 7)])
def test_sample_k_over_k2_device_equals_host_and_oracle(L, alpha, P):
    """exp(-k^2/4a)/k^2 proposal: the same draws on the device, on the host
    and in the oracle (modes bit for bit; weights carry S2, summed in another
    order by the oracle)."""
    p = rbe.make_params(L, alpha, 2.0, 1.0, P, seed=4321, kdist=rbe.KDIST_GAUSS_OVER_K2)
    for ev in (0, 5):
        mh, wh = rbe.sample_k(p, ev)
        md, wd = rbe.sample_k(p, ev, on_device=True)
        assert np.array_equal(mh, md.cpu().numpy()) and np.array_equal(wh, wd.cpu().numpy())
        mo, wo = oracle.sample_k(4321, ev, L, alpha, P, kdist=1)
        assert np.array_equal(mh, mo)
        assert np.allclose(wh, wo, rtol=1e-13, atol=0.0)


def test_forces_fp64_over_k2_modes(plain3k):
    """Forces with the library drawing exp(-k^2/4a)/k^2 modes itself match
    the oracle fed the oracle's draw of the same proposal."""
    p, s, _, _, _ = plain3k
    pk = dict(p, kdist=rbe.KDIST_GAUSS_OVER_K2)
    m, w = oracle.sample_k(p["seed"], 3, p["L"], p["alpha"], p["P"], kdist=1)
    ref = oracle_forces(pk, s, m, w, ev=3)
    F = gpu_forces(pk, s, m=None, w=None, ev=3)
    e = rel_err(F, ref["F"])
    print(f"plain3k FP64 over-k2 modes rel err {e:.3e}")
    assert e < TOL64


# ---------------------------------------------------------------------------
# binning
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,ncell", [(1, (3, 3, 3)), (777, (5, 4, 6)), (20000, (9, 9, 9)), (65537, (1, 2, 3))])
def test_build_cells_bit_exact(n, ncell):
    L = (n / 0.5) ** (1 / 3) if n > 1 else 3.0
    p = gen.preset("replica", n=n)
    s = gen.make_system(p) if n > 1 else dict(x=np.array([1.0]), y=np.array([2.0]), z=np.array([0.5]),
                                               q=np.array([0.0]), id=np.zeros(1, np.int32))
    L = p["L"] if n > 1 else 3.0
    x = s["x"].copy()
    if n > 5:  # boundary values: exactly 0, just below L, slightly negative, L itself, beyond L
        x[:5] = [0.0, L - 1e-13, -1e-18, L, 2 * L + 0.25]
    params = rbe.make_params(L, 0.3, 0.4 * L / 1.0 if n == 1 else 1.0, 0.5, 4, ncell=ncell)
    ctx = rbe.Context(params, n)
    t = lambda a: torch.as_tensor(a).cuda()  # noqa: E731
    cs, perm = ctx.build_cells(t(x), t(s["y"]), t(s["z"]), t(s["q"]))
    cs_o, perm_o = oracle.bin_cells(x, s["y"], s["z"], s["q"], L, ncell)
    assert np.array_equal(cs.cpu().numpy(), cs_o)
    assert np.array_equal(perm.cpu().numpy(), perm_o)
    ctx.close()


# ---------------------------------------------------------------------------
# FP64 forces: the 3k-ion configuration (all terms and each term alone)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def plain3k():
    p, s = system("plain3k")
    m, w = oracle.sample_k(p["seed"], 0, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w)
    return p, s, m, w, ref


def test_forces_fp64_plain3k_total_and_rho(plain3k):
    p, s, m, w, ref = plain3k
    F, re, im = gpu_forces(p, s, m=m, w=w, want_rho=True)
    assert rel_err(re, ref["rho_re"]) < TOL64 and rel_err(im, ref["rho_im"]) < TOL64
    e = rel_err(F, ref["F"])
    print(f"plain3k FP64 total rel err {e:.3e}, max row {max_row_err(F, ref['F']):.3e}")
    assert e < TOL64
    assert max_row_err(F, ref["F"]) < ROW64


@pytest.mark.parametrize("term,key", [(rbe.TERM_LJ, "lj"), (rbe.TERM_COUL_REAL, "coul"), (rbe.TERM_FOURIER, "fourier")])
def test_forces_fp64_plain3k_each_term(plain3k, term, key):
    p, s, m, w, ref = plain3k
    F = gpu_forces(p, s, terms=term, m=m, w=w)
    e = rel_err(F, ref[key])
    print(f"plain3k FP64 {key} rel err {e:.3e}")
    assert e < TOL64
    assert max_row_err(F, ref[key]) < ROW64


@pytest.mark.parametrize("ncell", [(3, 3, 3), (7, 7, 7), (13, 11, 12)])
def test_forces_fp64_independent_of_cell_grid(plain3k, ncell):
    p, s, m, w, ref = plain3k
    F = gpu_forces(p, s, m=m, w=w, ncell=ncell)
    assert rel_err(F, ref["F"]) < TOL64


def test_forces_fp64_device_drawn_modes_match(plain3k):
    p, s, m, w, ref = plain3k
    F = gpu_forces(p, s, m=None, w=None, ev=0)  # library draws the modes for eval 0 itself
    assert rel_err(F, ref["F"]) < TOL64


def test_forces_deterministic(plain3k):
    p, s, m, w, _ = plain3k
    F1 = gpu_forces(p, s, m=m, w=w)
    F2 = gpu_forces(p, s, m=m, w=w)
    assert np.array_equal(F1, F2)


# ---------------------------------------------------------------------------
# FP64 forces with the random batch list (electrolyte shape, 20k particles)
# ---------------------------------------------------------------------------
def test_forces_fp64_rbl_electrolyte_20k():
    p, s = system("electrolyte1m", n=20000)
    for ev in (0, 3):
        m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
        ref = oracle_forces(p, s, m, w, ev=ev, cells=False)
        F = gpu_forces(p, s, m=m, w=w, ev=ev)
        e = rel_err(F, ref["F"])
        print(f"electrolyte20k FP64 ev={ev} rel err {e:.3e}, max row {max_row_err(F, ref['F']):.3e}")
        assert e < TOL64
        assert max_row_err(F, ref["F"]) < ROW64
        assert np.abs(F.sum(axis=0)).max() < 1e-8 * np.abs(F).sum() / len(F)  # Eq. 12 + zero net Fourier force


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
@pytest.mark.parametrize("ghost", [0.0, 6.0])
def test_forces_rbl_charged_only_shell_20k(prec, tol, ghost):
    """Variant shell of charged particles only (r_lj <= r_core): the batches
    and the #S_i scaling follow the oracle's charged-only shell."""
    p, s = system("electrolyte1m", n=20000, rbl_shell=rbe.SHELL_CHARGED, ghost=ghost)
    m, w = oracle.sample_k(p["seed"], 2, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=2, cells=False)
    F = gpu_forces(p, s, prec=prec, m=m, w=w, ev=2)
    e = rel_err(F, ref["F"])
    print(f"electrolyte20k charged-only shell prec={prec} ghost={ghost} rel err {e:.3e}")
    assert e < tol
    # the literal shell gives a different estimate on the same draw
    p0 = dict(p, rbl_shell=rbe.SHELL_ALL)
    assert rel_err(gpu_forces(p0, s, prec=prec, m=m, w=w, ev=2), F) > 1e-6


def test_forces_fp64_rbl_small_box_wrapping_stencil():
    """Fewer than 2s+1 cells per axis: stencil rows revisit cells with other images."""
    p, s = system("electrolyte1m", n=1500)  # L = 12.3, r_coul = 6
    m, w = oracle.sample_k(p["seed"], 1, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=1, cells=False)
    for ncell in ((0, 0, 0), (2, 2, 2), (1, 1, 1), (5, 3, 4)):
        F = gpu_forces(p, s, m=m, w=w, ev=1, ncell=ncell)
        assert rel_err(F, ref["F"]) < TOL64, ncell


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
@pytest.mark.parametrize("xsplit", [3, 6])
def test_forces_rbl_electrolyte_20k_split_x(prec, tol, xsplit):
    """Cells split along x only (stencil radii differ per axis): same forces."""
    p, s = system("electrolyte1m", n=20000)
    m, w = oracle.sample_k(p["seed"], 5, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=5, cells=False)
    nc = int(p["L"] // 3.0)
    F = gpu_forces(p, s, prec=prec, m=m, w=w, ev=5, ncell=(xsplit * nc, nc, nc))
    e = rel_err(F, ref["F"])
    print(f"electrolyte20k split x{xsplit} prec={prec} rel err {e:.3e}")
    assert e < tol


# ---------------------------------------------------------------------------
# FP32-compensated form
# ---------------------------------------------------------------------------
def test_forces_fp32c_plain3k(plain3k):
    p, s, m, w, ref = plain3k
    for term, key in ((rbe.TERM_LJ, "lj"), (rbe.TERM_COUL_REAL, "coul"), (rbe.TERM_FOURIER, "fourier"),
                      (rbe.TERM_ALL, "F")):
        F = gpu_forces(p, s, prec=rbe.FP32C, terms=term, m=m, w=w)
        e = rel_err(F, ref[key])
        print(f"plain3k FP32C {key} rel err {e:.3e}, max row {max_row_err(F, ref[key]):.3e}")
        assert e < TOL32
        assert max_row_err(F, ref[key]) < ROW32


def test_forces_fp32c_rbl_electrolyte_20k():
    p, s = system("electrolyte1m", n=20000)
    m, w = oracle.sample_k(p["seed"], 2, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=2, cells=False)
    F = gpu_forces(p, s, prec=rbe.FP32C, m=m, w=w, ev=2)
    e = rel_err(F, ref["F"])
    print(f"electrolyte20k FP32C rel err {e:.3e}, max row {max_row_err(F, ref['F']):.3e}")
    assert e < TOL32
    assert max_row_err(F, ref["F"]) < ROW32


# ---------------------------------------------------------------------------
# velocity Verlet: 10 steps of the 3k configuration
# ---------------------------------------------------------------------------
def test_step_fp64_plain3k_trajectory():
    p, s = system("plain3k")
    n = p["n"]
    params = rbe.params_from_preset(p)
    ctx = rbe.Context(params, n)
    st = to_device(s)
    ctx.forces(st, None, None, 0)  # eval 0: initial force
    ctx.step(st, 10, 1)
    torch.cuda.synchronize()
    ctx.sync_check()
    ids = st.id.cpu().numpy()
    assert np.array_equal(np.sort(ids), np.arange(n))
    # oracle trajectory (eval e draws its own modes)
    osys = oracle.sys_from_preset(p)
    r = np.stack([s["x"], s["y"], s["z"]], axis=1)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)

    def force(r, ev):
        m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
        return oracle.total_force(r[:, 0], r[:, 1], r[:, 2], s["q"], s["id"], osys, m, w, seed=p["seed"], ev=ev)["F"]

    F = force(r, 0)
    for k in range(10):
        v = oracle.kick(F, v, p["dt"] / 2)
        r = oracle.drift_wrap(r, v, p["dt"], p["L"])
        F = force(r, k + 1)
        v = oracle.kick(F, v, p["dt"] / 2)
    gx = np.empty((n, 3)); gv = np.empty((n, 3)); gf = np.empty((n, 3))
    gx[ids] = np.stack([st.x.cpu().numpy(), st.y.cpu().numpy(), st.z.cpu().numpy()], axis=1)
    gv[ids] = np.stack([st.vx.cpu().numpy(), st.vy.cpu().numpy(), st.vz.cpu().numpy()], axis=1)
    gf[ids] = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    d = (gx - r + p["L"] / 2) % p["L"] - p["L"] / 2
    assert np.abs(d).max() < 1e-12 * p["L"]
    assert rel_err(gv, v) < TOL64
    assert rel_err(gf, F) < TOL64
    ctx.close()


# ---------------------------------------------------------------------------
# errors reported through the ABI
# ---------------------------------------------------------------------------
def test_non_neutral_rejected(plain3k):
    """Neutrality (Eq. 1) and finite charges are checked on the device (no
    call waits for them): rbe_sync_check reports the flag."""
    p, s, m, w, _ = plain3k
    s2 = dict(s)
    s2["q"] = s["q"].copy()
    s2["q"][0] = 0.0
    with pytest.raises(rbe.RbeError) as e:
        gpu_forces(p, s2, m=m, w=w)
    assert e.value.code == rbe.RBE_ENONNEUTRAL
    params = rbe.params_from_preset(p)
    ctx = rbe.Context(params, p["n"])
    st = to_device(s2)
    ctx.step(st, 2, 1)
    with pytest.raises(rbe.RbeError) as e:
        ctx.sync_check()
    assert e.value.code == rbe.RBE_ENONNEUTRAL
    st = to_device(s)
    st.q[7] = float("nan")
    ctx.forces(st, None, None, 0)
    with pytest.raises(rbe.RbeError) as e:
        ctx.sync_check()
    assert e.value.code == rbe.RBE_ENONFINITE
    ctx.close()


def test_capacity_and_nonfinite_reported(plain3k):
    p, s, m, w, _ = plain3k
    params = rbe.params_from_preset(p)
    ctx = rbe.Context(params, 100)
    with pytest.raises(rbe.RbeError) as e:
        ctx.forces(to_device(s), None, None, 0)
    assert e.value.code == rbe.RBE_ERANGE
    ctx.close()
    ctx = rbe.Context(params, p["n"])
    st = to_device(s)
    ctx.forces(st, None, None, 0)
    st.vx[5] = float("nan")
    ctx.step(st, 1, 1)
    with pytest.raises(rbe.RbeError) as e:
        ctx.sync_check()
    assert e.value.code == rbe.RBE_ENONFINITE
    ctx.close()


# ---------------------------------------------------------------------------
# ghost shell: the padded, non-periodic traversal equals the periodic sums
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
def test_forces_ghost_shell_matches_periodic(prec, tol):
    p, s = system("subdomain64m", n=40000)  # L = 36.8, ghost width 6
    m, w = oracle.sample_k(p["seed"], 0, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, cells=True)
    F = gpu_forces(p, s, prec=prec, m=m, w=w)
    e = rel_err(F, ref["F"])
    print(f"ghost shell 40k prec={prec} rel err {e:.3e}")
    assert e < tol
    # same result as the periodic traversal of the same system
    pp = dict(p)
    pp["ghost"] = 0.0
    F2 = gpu_forces(pp, s, prec=prec, m=m, w=w)
    assert rel_err(F, F2) < (1e-13 if prec == rbe.FP64 else 1e-6)


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
def test_forces_ghost_shell_split_x(prec, tol):
    """Ghost layers per axis sized for per-axis stencil radii (x cells 4x finer)."""
    p, s = system("subdomain64m", n=40000)
    m, w = oracle.sample_k(p["seed"], 2, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=2, cells=True)
    nc = int(p["L"] // 2.5)
    F = gpu_forces(p, s, prec=prec, m=m, w=w, ev=2, ncell=(4 * nc, nc, nc))
    e = rel_err(F, ref["F"])
    print(f"ghost shell split x prec={prec} rel err {e:.3e}")
    assert e < tol


def test_forces_ghost_shell_with_random_batch_list():
    p, s = system("electrolyte1m", n=20000, ghost=6.0)
    m, w = oracle.sample_k(p["seed"], 4, p["L"], p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=4, cells=False)
    F = gpu_forces(p, s, m=m, w=w, ev=4)
    e = rel_err(F, ref["F"])
    print(f"ghost shell + list 20k rel err {e:.3e}")
    assert e < TOL64


@pytest.mark.parametrize("ghost", [0.0, 6.0])
def test_step_random_batch_list_fp64(ghost):
    """Several steps with the random batch list: after the first step the id
    -> slot map of the batch members comes from the reorder; the final forces
    must equal a fresh oracle evaluation at the final positions."""
    p, s = system("electrolyte1m", n=20000, ghost=ghost)
    params = rbe.params_from_preset(p, prec=rbe.FP64)
    ctx = rbe.Context(params, p["n"])
    st = to_device(s)
    ctx.forces(st, None, None, 0)
    ctx.step(st, 4, 1)
    torch.cuda.synchronize()
    ctx.sync_check()
    x = st.x.cpu().numpy(); y = st.y.cpu().numpy(); z = st.z.cpu().numpy()
    q = st.q.cpu().numpy(); ids = st.id.cpu().numpy()
    m, w = oracle.sample_k(p["seed"], 4, p["L"], p["alpha"], p["P"])
    ref = oracle.total_force(x, y, z, q, ids, oracle.sys_from_preset(p), m, w, seed=p["seed"], ev=4, cells=False,
                             components=False)["F"]
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    e = rel_err(F, ref)
    print(f"RBL 4 steps ghost={ghost} final-force rel err {e:.3e}")
    assert e < TOL64
    ctx.close()


def test_step_ghost_shell_fp32c():
    p, s = system("subdomain64m", n=30000)
    params = rbe.params_from_preset(p, prec=rbe.FP32C)
    ctx = rbe.Context(params, p["n"])
    st = to_device(s)
    ctx.forces(st, None, None, 0)
    ctx.step(st, 5, 1)
    torch.cuda.synchronize()
    ctx.sync_check()
    # the final force equals a fresh evaluation at the final positions (eval 5)
    x = st.x.cpu().numpy(); y = st.y.cpu().numpy(); z = st.z.cpu().numpy()
    q = st.q.cpu().numpy(); ids = st.id.cpu().numpy()
    m, w = oracle.sample_k(p["seed"], 5, p["L"], p["alpha"], p["P"])
    ref = oracle.total_force(x, y, z, q, ids, oracle.sys_from_preset(p), m, w, seed=p["seed"], ev=5, cells=True,
                             components=False)["F"]
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    assert rel_err(F, ref) < TOL32
    ctx.close()


# ---------------------------------------------------------------------------
# exact boundaries: lattice distances equal to the cutoffs, particles on cell
# faces (the trimmed stencil rows and the core/shell split must keep every
# pair the oracle keeps)
# ---------------------------------------------------------------------------
def lattice_with_vacancies(seed=7, a=1.25, n=12, frac_removed=0.1):
    """Rock-salt charges on a simple cubic lattice of spacing a (all
    coordinates exact binary fractions), with an equal number of + and -
    sites removed so that the forces do not cancel by symmetry."""
    rng = np.random.default_rng(seed)
    g = np.arange(n) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    ijk = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    q = np.where(ijk.sum(1) % 2 == 0, 1.0, -1.0)
    keep = np.ones(len(q), bool)
    k = int(frac_removed * len(q) / 2)
    keep[rng.choice(np.nonzero(q > 0)[0], k, replace=False)] = False
    keep[rng.choice(np.nonzero(q < 0)[0], k, replace=False)] = False
    s = dict(x=X.ravel()[keep].copy(), y=Y.ravel()[keep].copy(), z=Z.ravel()[keep].copy(), q=q[keep].copy())
    s["id"] = np.arange(len(s["q"]), dtype=np.int32)
    return s, n * a


@pytest.mark.parametrize("ncell", [(6, 6, 6), (4, 4, 4), (12, 12, 12), (24, 6, 6), (18, 4, 4)])
def test_forces_fp64_cutoffs_on_lattice_distances(ncell):
    s, L = lattice_with_vacancies()
    # r_lj = 2a, r_coul = 4a: many pairs exactly at each cutoff
    p = dict(seed=77, n=len(s["q"]), L=L, alpha=0.3, r_coul=5.0, r_lj=2.5, r_core=0.0, p_shell=0, P=40, dt=0.002,
             ghost=0.0)
    m, w = oracle.sample_k(p["seed"], 0, L, p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=0, cells=False)
    for term, key in ((rbe.TERM_LJ, "lj"), (rbe.TERM_COUL_REAL, "coul"), (rbe.TERM_ALL, "F")):
        F = gpu_forces(p, s, terms=term, m=m, w=w, ncell=ncell)
        assert rel_err(F, ref[key]) < TOL64, (ncell, key)


@pytest.mark.parametrize("ncell", [(6, 6, 6), (4, 4, 4), (24, 6, 6)])
def test_forces_fp64_rbl_core_on_lattice_distance(ncell):
    s, L = lattice_with_vacancies(seed=8)
    # r_core = 3a exactly, shell out to r_coul = 4a; p below the shell size
    p = dict(seed=78, n=len(s["q"]), L=L, alpha=0.3, r_coul=5.0, r_lj=2.5, r_core=3.75, p_shell=8, P=40,
             dt=0.002, ghost=0.0)
    m, w = oracle.sample_k(p["seed"], 3, L, p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, ev=3, cells=False)
    F = gpu_forces(p, s, m=m, w=w, ev=3, ncell=ncell)
    assert rel_err(F, ref["F"]) < TOL64, ncell


# ---------------------------------------------------------------------------
# degenerate sizes: two particles, almost no charges, one mode, ragged counts
# ---------------------------------------------------------------------------
def small_system(n, n_charged, L, seed):
    rng = np.random.default_rng(seed)
    s = dict(x=rng.uniform(0, L, n), y=rng.uniform(0, L, n), z=rng.uniform(0, L, n), q=np.zeros(n))
    s["q"][: n_charged // 2] = 1.0
    s["q"][n_charged // 2: n_charged] = -1.0
    s["id"] = rng.permutation(n).astype(np.int32)
    return s


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
@pytest.mark.parametrize("n,n_charged,r_core,p_shell,P", [
    (2, 2, 0.0, 0, 1),        # one ion pair, one mode
    (2, 2, 1.5, 4, 3),        # random batch list with at most one shell member
    (67, 2, 1.5, 4, 5),       # ragged count, two charges among neutrals
    (300, 0, 0.0, 0, 4),      # no charges at all: LJ only, Fourier part empty
    (301, 300, 2.0, 8, 7),    # ragged, one neutral
])
def test_forces_degenerate_sizes(prec, tol, n, n_charged, r_core, p_shell, P):
    L = 12.0
    s = small_system(n, n_charged, L, seed=n + P)
    # keep particles apart so LJ stays finite
    s["x"] = (np.arange(n) % 7) * (L / 7) + 0.3 * (s["x"] / L)
    s["y"] = ((np.arange(n) // 7) % 7) * (L / 7) + 0.3 * (s["y"] / L)
    s["z"] = (np.arange(n) // 49) * (L / 7) + 0.3 * (s["z"] / L)
    p = dict(seed=91 + n, n=n, L=L, alpha=0.4, r_coul=5.0, r_lj=2.5, r_core=r_core, p_shell=p_shell, P=P,
             dt=0.002, ghost=0.0)
    print(f"degenerate n={n} nq={n_charged} r_core={r_core} P={P} prec={prec}", flush=True)
    m, w = oracle.sample_k(p["seed"], 2, L, p["alpha"], P)
    ref = oracle_forces(p, s, m, w, ev=2, cells=False)
    F = gpu_forces(p, s, prec=prec, m=m, w=w, ev=2)
    assert np.all(np.isfinite(F))
    assert rel_err(F, ref["F"]) < tol


# ---------------------------------------------------------------------------
# near-field tiles: a halo denser than the staging is processed in row chunks
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, TOL32)])
@pytest.mark.parametrize("ghost", [0.0, 6.0])
def test_forces_dense_cluster_in_sparse_box(prec, tol, ghost):
    """All particles packed (minimum separation 0.55) into a 9-sigma cube of a
    40-sigma box: tiles sized for the mean density meet halos tens of times
    denser, which they stage in chunks of rows; forces still match."""
    L, n = 40.0, 2000
    x, y, z = gen.rsa_positions(77, 0, n, [9.0, 9.0, 9.0], dmin=0.55)
    q = gen.charges(77, 0, n, 150, 150)
    s = dict(x=x + 15.0, y=y + 15.5, z=z + 16.0, q=q, id=np.arange(n, dtype=np.int32),
             L=np.array([L, L, L]))
    p = dict(seed=77, n=n, L=L, alpha=0.3, r_coul=6.0, r_lj=2.5, r_core=0.0, p_shell=0, P=50, dt=0.002,
             ghost=ghost)
    m, w = oracle.sample_k(p["seed"], 0, L, p["alpha"], p["P"])
    ref = oracle_forces(p, s, m, w, cells=False)
    for ncell in ((0, 0, 0), (64, 16, 16)):
        F = gpu_forces(p, s, prec=prec, m=m, w=w, ncell=ncell)
        e, r = rel_err(F, ref["F"]), max_row_err(F, ref["F"])
        print(f"dense cluster prec={prec} ghost={ghost} ncell={ncell}: rel err {e:.3e}, max row {r:.3e}")
        assert e < tol and r < (ROW64 if prec == rbe.FP64 else ROW32)


def test_tile_row_beyond_the_staging_is_reported():
    """One y/z cell row packed far above the mean density (about 1,840 records
    in a tile's halo row, where the tile's staging holds about 1,350 at this
    mean density): the row cannot be staged, the kernel leaves it out and
    rbe_sync_check reports RBE_ERANGE instead of returning incomplete forces
    silently."""
    # cells of 0.628 x 2.51 x 2.51: the LJ stencil is 4 x 1 x 1 cells
    L, ncell = 20.1, (32, 8, 8)
    bx, by, bz = gen.rsa_positions(91, 0, 2400, [L, L, L], dmin=0.8)
    # the row of y/z cell (2, 2): y, z in [5, 7.5)
    keep = ~((by >= 4.6) & (by < 7.9) & (bz >= 4.6) & (bz < 7.9))
    rx, ry, rz = gen.rsa_positions(92, 0, 1900, [L, 2.4, 2.4], dmin=0.3)
    x = np.concatenate([bx[keep], rx])
    y = np.concatenate([by[keep], ry + 5.05])
    z = np.concatenate([bz[keep], rz + 5.05])
    n = len(x)
    nq = 100
    q = np.zeros(n)
    q[:nq] = 1.0
    q[nq:2 * nq] = -1.0
    s = dict(x=x, y=y, z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), q=q,
             id=np.arange(n, dtype=np.int32), L=np.array([L, L, L]))
    params = rbe.make_params(L, 0.35, 6.0, 2.5, 50, prec=rbe.FP32C, ncell=ncell)
    ctx = rbe.Context(params, n)
    st = to_device(s)
    print(f"dense row: n={n}, {len(rx)} in one cell row", flush=True)
    ctx.forces(st, None, None, 0)
    torch.cuda.synchronize()
    with pytest.raises(rbe.RbeError) as e:
        ctx.sync_check()
    assert e.value.code == rbe.RBE_ERANGE and "LDS staging" in str(e.value)
    ctx.close()
