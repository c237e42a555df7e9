"""rbe_forces_noalloc (no context, no device allocation: the library's
file-scope scratch array) against rbe_forces on a context with the same
parameters, through the C ABI, on two calls in a row, the second with a
smaller input than the first."""
import numpy as np
import pytest

import oracle
from gpu_common import max_row_err, rel_err, system, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_02694_amd as rbe  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


def host_f(st):
    return np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)


def ctx_forces(p, s, prec, m, w, ev):
    ctx = rbe.Context(rbe.params_from_preset(p, prec=prec), p["n"])
    st = to_device(s)
    rho = torch.zeros(2 * p["P"], dtype=torch.float64, device="cuda")
    ctx.forces(st, m, w, ev, rho)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = host_f(st)
    ctx.close()
    return F, rho.cpu().numpy()


@pytest.mark.parametrize("prec,tol", [(rbe.FP64, 1e-12), (rbe.FP32C, 1e-5)])
def test_noalloc_matches_context_two_calls(prec, tol):
    """First the 20k electrolyte (random batch list, Eq. 12), then a smaller
    3k system of another shape on the same scratch: both equal the context
    path (FP64 to 1e-12, FP32C to 1e-5; the structure-factor partials are
    chunked differently), and the second call is not disturbed by what the
    first left in the array."""
    cases = [system("electrolyte1m", n=20000), system("plain3k")]
    for k, (p, s) in enumerate(cases):
        assert p["n"] <= rbe.NOALLOC_MAX_N
        ev = 2 + k
        mh, wh = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
        m = torch.as_tensor(mh.ravel()).cuda()
        w = torch.as_tensor(wh).cuda()
        ref, rho_ref = ctx_forces(p, s, prec, m, w, ev)
        st = to_device(s)
        rho = torch.zeros(2 * p["P"], dtype=torch.float64, device="cuda")
        status = torch.full((1,), -99, dtype=torch.int32, device="cuda")
        print(f"noalloc call {k}: n={p['n']} prec={prec}", flush=True)
        rbe.forces_noalloc(rbe.params_from_preset(p, prec=prec), st, m, w, ev, rho, status)
        torch.cuda.synchronize()
        assert int(status.item()) == rbe.RBE_OK
        F = host_f(st)
        e = rel_err(F, ref)
        print(f"  rel err vs context {e:.3e}, max row {max_row_err(F, ref):.3e}")
        assert e < tol
        assert rel_err(rho.cpu().numpy(), rho_ref) < (1e-13 if prec == rbe.FP64 else 1e-6)


def test_noalloc_limits_and_device_status():
    p, s = system("plain3k")
    m, w = oracle.sample_k(p["seed"], 0, p["L"], p["alpha"], p["P"])
    md = torch.as_tensor(m.ravel()).cuda()
    wd = torch.as_tensor(w).cuda()
    st = to_device(s)
    with pytest.raises(rbe.RbeError) as e:
        rbe.forces_noalloc(rbe.params_from_preset(p), st, None, None, 0)
    assert e.value.code == rbe.RBE_EINVAL
    with pytest.raises(rbe.RbeError) as e:
        rbe.forces_noalloc(rbe.params_from_preset(dict(p, P=rbe.NOALLOC_MAX_P + 1)), st, md, wd, 0)
    assert e.value.code == rbe.RBE_ERANGE
    q = s["q"].copy()
    q[0] = 0.0  # not neutral: reported through the device status
    st2 = to_device(dict(s, q=q))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    rbe.forces_noalloc(rbe.params_from_preset(p), st2, md, wd, 0, None, status)
    torch.cuda.synchronize()
    assert int(status.item()) == rbe.RBE_ENONNEUTRAL
    # the next call starts from a clear flag
    rbe.forces_noalloc(rbe.params_from_preset(p), st, md, wd, 0, None, status)
    torch.cuda.synchronize()
    assert int(status.item()) == rbe.RBE_OK
