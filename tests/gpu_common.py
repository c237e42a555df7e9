"""Helpers shared by the GPU parity tests (inputs from ``gen``, references from ``oracle``)."""
import numpy as np

import gen
import oracle
import paper_2609_02694_amd as rbe


def rel_err(a, b):
    """RMS relative error ||a - b||_2 / ||b||_2 over all particles and components."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def max_row_err(a, b):
    """Largest per-particle error |a_i - b_i| (Euclidean over components) in
    units of the RMS particle force of b: one bad row cannot hide in the RMS."""
    a = np.asarray(a, np.float64).reshape(-1, 3)
    b = np.asarray(b, np.float64).reshape(-1, 3)
    frms = np.sqrt((b ** 2).sum() / len(b))
    return float(np.sqrt(((a - b) ** 2).sum(axis=1)).max() / (frms if frms > 0 else 1.0))


# Per-row bounds (in units of the RMS particle force) beside the RMS bounds:
# FP64 rows agree to about 1e-13 of the RMS force; FP32C rows carry the
# single-precision rounding of up to ~100 pair terms scaled by the largest
# forces (a few times the RMS), measured up to a few 1e-6.
ROW64 = 1e-10
ROW32 = 2e-4


def system(name, n=None, **over):
    p = gen.preset(name, n=n, **over)
    return p, gen.make_system(p)


def to_device(s):
    return rbe.Particles.from_numpy(s)


def gpu_forces(p, s, prec=rbe.FP64, terms=rbe.TERM_ALL, ev=0, m=None, w=None, ncell=(0, 0, 0), want_rho=False):
    import torch
    params = rbe.params_from_preset(p, prec=prec, terms=terms, ncell=ncell)
    ctx = rbe.Context(params, len(s["x"]))
    st = to_device(s)
    md = wd = None
    if m is not None:
        md = torch.as_tensor(np.ascontiguousarray(m, np.int32).ravel()).cuda()
        wd = torch.as_tensor(np.ascontiguousarray(w, np.float64)).cuda()
    rho = torch.zeros(2 * p["P"], dtype=torch.float64, device="cuda") if want_rho else None
    ctx.forces(st, md, wd, ev, rho)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    ctx.close()
    if want_rho:
        r = rho.cpu().numpy()
        return F, r[: p["P"]], r[p["P"]:]
    return F


def oracle_forces(p, s, m, w, ev=0, terms=oracle.LJ | oracle.COUL_REAL | oracle.FOURIER, cells=None):
    osys = oracle.sys_from_preset(p)
    return oracle.total_force(s["x"], s["y"], s["z"], s["q"], s["id"], osys, m, w, seed=p["seed"], ev=ev,
                              terms=terms, cells=cells)
