"""GPU parity of the Nose-Hoover NVT step (rbe_step with nvt_tau > 0).

Trajectories through the C ABI against the oracle's NVT step on the same
seeded inputs: positions to 1e-12 L, velocities and forces to 1e-12 RMS
relative, the thermostat variables xi and eta to 1e-12 relative. A
thermostat of infinite mass must reproduce the NVE step bit for bit.
"""
import numpy as np
import pytest

import oracle
from gpu_common import rel_err, system, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_02694_amd as rbe  # noqa: E402

TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


def _gather(st, ids, n):
    out = {}
    for key, names in (("x", ("x", "y", "z")), ("v", ("vx", "vy", "vz")), ("f", ("fx", "fy", "fz"))):
        a = np.empty((n, 3))
        a[ids] = np.stack([getattr(st, k).cpu().numpy() for k in names], axis=1)
        out[key] = a
    return out


def _run_gpu(p, s, nsteps, nh0=(0.0, 0.0), split=None):
    ctx = rbe.Context(rbe.params_from_preset(p), p["n"])
    st = to_device(s)
    st.nh = torch.tensor(nh0, dtype=torch.float64, device="cuda")
    ctx.forces(st, None, None, 0)
    done = 0
    for k in (split or [nsteps]):
        ctx.step(st, k, 1 + done)
        done += k
    torch.cuda.synchronize()
    ctx.sync_check()
    ids = st.id.cpu().numpy()
    out = _gather(st, ids, p["n"])
    out["nh"] = st.nh.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("split", [None, [3, 7]])
def test_step_nvt_fp64_plain3k_trajectory(split):
    """Ten NVT steps (one call, or two calls of 3 and 7 steps) against the
    oracle's trajectory; the thermostat starts off its equilibrium (kT below
    the initial temperature) so xi moves."""
    p, s = system("plain3k", nvt_kT=0.6, nvt_tau=0.05)
    n, nsteps = p["n"], 10
    g = _run_gpu(p, s, nsteps, nh0=(0.1, 0.0), split=split)
    osys = oracle.sys_from_preset(p)

    def force(r, ev):
        m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
        return oracle.total_force(r[:, 0], r[:, 1], r[:, 2], s["q"], s["id"], osys, m, w, seed=p["seed"],
                                  ev=ev)["F"]

    r = np.stack([s["x"], s["y"], s["z"]], axis=1)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)
    F = force(r, 0)
    xi, eta = 0.1, 0.0
    for k in range(nsteps):
        r, v, F, xi, eta = oracle.nvt_step(r, v, F, xi, eta, lambda rr: force(rr, k + 1), p["dt"], p["L"], 1.0,
                                           p["nvt_kT"], p["nvt_tau"])
    d = (g["x"] - r + p["L"] / 2) % p["L"] - p["L"] / 2
    print(f"NVT 10 steps: xi {g['nh'][0]:.12e} (oracle {xi:.12e}), v rel {rel_err(g['v'], v):.2e}")
    assert abs(xi - 0.1) > 1e-3
    assert np.abs(d).max() < 1e-12 * p["L"]
    assert rel_err(g["v"], v) < TOL64
    assert rel_err(g["f"], F) < TOL64
    assert abs(g["nh"][0] - xi) < TOL64 * abs(xi) and abs(g["nh"][1] - eta) < TOL64 * abs(eta)


def test_step_nvt_infinite_thermostat_mass_equals_nve_bitwise():
    """With an effectively infinite thermostat mass every velocity scaling is
    exactly 1: the NVT launches must reproduce the fused NVE step bit for bit
    (random batch list on, so the Eq. 12 mean goes through both paths)."""
    p, s = system("electrolyte1m", n=20000)
    nve = _run_gpu(p, s, 5)
    pn = dict(p, nvt_kT=1.0, nvt_tau=1e12)
    nvt = _run_gpu(pn, s, 5)
    assert abs(nvt["nh"][0]) < 1e-20
    for key in ("x", "v", "f"):
        assert np.array_equal(nve[key], nvt[key]), key


def test_step_nvt_random_batch_list_final_force():
    """Four NVT steps with the random batch list: the final forces equal a
    fresh oracle evaluation at the final positions, and the thermostat moved."""
    p, s = system("electrolyte1m", n=20000, nvt_kT=0.5, nvt_tau=0.02)
    ctx = rbe.Context(rbe.params_from_preset(p), p["n"])
    st = to_device(s)
    st.nh = torch.zeros(2, dtype=torch.float64, device="cuda")
    ctx.forces(st, None, None, 0)
    ctx.step(st, 4, 1)
    torch.cuda.synchronize()
    ctx.sync_check()
    x = st.x.cpu().numpy(); y = st.y.cpu().numpy(); z = st.z.cpu().numpy()
    q = st.q.cpu().numpy(); ids = st.id.cpu().numpy()
    m, w = oracle.sample_k(p["seed"], 4, p["L"], p["alpha"], p["P"])
    ref = oracle.total_force(x, y, z, q, ids, oracle.sys_from_preset(p), m, w, seed=p["seed"], ev=4,
                             components=False)["F"]
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    assert rel_err(F, ref) < TOL64
    xi = float(st.nh[0].cpu())
    assert xi != 0.0 and np.isfinite(xi)
    ctx.close()


def test_nvt_errors():
    p, s = system("plain3k", n=500, L=17.0, nvt_kT=1.0, nvt_tau=0.1)
    ctx = rbe.Context(rbe.params_from_preset(p), p["n"])
    st = to_device(s)  # no thermostat state
    with pytest.raises(rbe.RbeError):
        ctx.step(st, 1, 1)
    ctx.close()
    bad = dict(p, nvt_kT=0.0)
    with pytest.raises(rbe.RbeError):
        rbe.Context(rbe.params_from_preset(bad), p["n"])
    pr = rbe.params_from_preset(dict(p, n=2000, L=26.0))
    with pytest.raises(rbe.RbeError):
        rbe.Context.batch([pr, pr], [0, 2000, 4000])


@pytest.fixture(scope="module")
def ljel20k():
    """The paper's LJ electrolyte (one short-range cutoff r_s = 8 for LJ and
    Coulomb, core 4, p = 30, P = 200, dt = 0.001, Nose-Hoover at kT = 1) at
    20,000 ions and the paper's density."""
    p, s = system("ljelectrolyte", n=20000)
    m, w = oracle.sample_k(p["seed"], 0, p["L"], p["alpha"], p["P"])
    ref = oracle.total_force(s["x"], s["y"], s["z"], s["q"], s["id"], oracle.sys_from_preset(p), m, w,
                             seed=p["seed"], ev=0, components=False)
    return p, s, m, w, ref


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, TOL64), (rbe.FP32C, 1e-5)])
def test_forces_ljelectrolyte_20k(ljel20k, prec, tol):
    from gpu_common import gpu_forces
    p, s, m, w, ref = ljel20k
    F = gpu_forces(p, s, prec=prec, m=m, w=w)
    e = rel_err(F, ref["F"])
    print(f"LJ electrolyte 20k prec={prec} rel err {e:.3e}")
    assert e < tol


def test_step_nvt_ljelectrolyte_20k_trajectory(ljel20k):
    p, s, _, _, _ = ljel20k
    nsteps = 3
    g = _run_gpu(p, s, nsteps)
    osys = oracle.sys_from_preset(p)

    def force(r, ev):
        m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
        return oracle.total_force(r[:, 0], r[:, 1], r[:, 2], s["q"], s["id"], osys, m, w, seed=p["seed"], ev=ev,
                                  components=False)["F"]

    r = np.stack([s["x"], s["y"], s["z"]], axis=1)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)
    F = force(r, 0)
    xi, eta = 0.0, 0.0
    for k in range(nsteps):
        r, v, F, xi, eta = oracle.nvt_step(r, v, F, xi, eta, lambda rr: force(rr, k + 1), p["dt"], p["L"], 1.0,
                                           p["nvt_kT"], p["nvt_tau"])
    d = (g["x"] - r + p["L"] / 2) % p["L"] - p["L"] / 2
    print(f"LJ electrolyte NVT: xi {g['nh'][0]:.12e} (oracle {xi:.12e}), v rel {rel_err(g['v'], v):.2e}")
    assert np.abs(d).max() < 1e-12 * p["L"]
    assert rel_err(g["v"], v) < TOL64
    assert rel_err(g["f"], F) < TOL64
    assert abs(g["nh"][0] - xi) <= TOL64 * abs(xi) + 1e-15 and abs(g["nh"][1] - eta) <= TOL64 * abs(eta) + 1e-18


def test_step_nvt_ghost_shell_fp32c_tracks_fp64():
    """NVT on a ghost-shell context in FP32C: after 4 steps the forces match a
    fresh oracle evaluation to the FP32C bound and the thermostat variable
    follows the FP64 run to the size of the FP32C force error."""
    p, s = system("subdomain64m", n=30000, nvt_kT=0.8, nvt_tau=0.05)
    out = {}
    for prec in (rbe.FP64, rbe.FP32C):
        ctx = rbe.Context(rbe.params_from_preset(p, prec=prec), p["n"])
        st = to_device(s)
        st.nh = torch.zeros(2, dtype=torch.float64, device="cuda")
        ctx.forces(st, None, None, 0)
        ctx.step(st, 4, 1)
        torch.cuda.synchronize()
        ctx.sync_check()
        out[prec] = (st, float(st.nh[0].cpu()))
        ctx.close()
    st, xi32 = out[rbe.FP32C]
    xi64 = out[rbe.FP64][1]
    x = st.x.cpu().numpy(); y = st.y.cpu().numpy(); z = st.z.cpu().numpy()
    q = st.q.cpu().numpy(); ids = st.id.cpu().numpy()
    m, w = oracle.sample_k(p["seed"], 4, p["L"], p["alpha"], p["P"])
    ref = oracle.total_force(x, y, z, q, ids, oracle.sys_from_preset(p), m, w, seed=p["seed"], ev=4, cells=True,
                             components=False)["F"]
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    assert rel_err(F, ref) < 1e-5
    assert xi64 != 0.0 and abs(xi32 - xi64) < 1e-6 * abs(xi64)
