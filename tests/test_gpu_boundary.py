"""The boundary's contract on the GPU: rbe_step never waits for the device
(so it can be captured in a HIP graph and replayed), its result does not
depend on how the steps are split over calls, and the FP64 path with the
random batch list is deterministic bit for bit.
"""
import numpy as np
import pytest

from gpu_common import system, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_02694_amd as rbe  # noqa: E402

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "q", "id")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


def snapshot(st):
    return {k: getattr(st, k).clone() for k in FIELDS}


def restore(st, snap):
    for k in FIELDS:
        getattr(st, k).copy_(snap[k])


def by_id(st):
    """State arrays indexed by particle id (the step returns cell order)."""
    ids = st.id.cpu().numpy()
    out = {}
    for k in FIELDS:
        a = getattr(st, k).cpu().numpy()
        b = np.empty_like(a)
        b[ids] = a
        out[k] = b
    return out


def assert_same_bits(a, b):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


CASES = [
    ("electrolyte1m", 20_000, rbe.FP64),   # random batch list, Eq. 12
    ("electrolyte1m", 20_000, rbe.FP32C),
    ("plain3k", None, rbe.FP64),
    ("subdomain64m", 40_000, rbe.FP32C),   # ghost shell
]


@pytest.mark.parametrize("name,n,prec", CASES)
def test_step_split_over_calls_is_bit_identical(name, n, prec):
    """k + (N - k) steps in two calls equal N steps in one call (ids map the
    particles: each call returns cell order), and running the same steps
    twice gives the same bits (deterministic with the random batch list)."""
    p, s = system(name, n=n)
    print(f"{name} n={p['n']} prec={prec}", flush=True)
    ctx = rbe.Context(rbe.params_from_preset(p, prec=prec), p["n"])
    st = to_device(s)
    ctx.forces(st, None, None, 0)
    start = snapshot(st)
    ctx.step(st, 5, 1)
    one = by_id(st)
    restore(st, start)
    ctx.step(st, 5, 1)
    assert_same_bits(by_id(st), one)
    restore(st, start)
    ctx.step(st, 2, 1)
    ctx.step(st, 3, 3)
    assert_same_bits(by_id(st), one)
    restore(st, start)
    ctx.step(st, 1, 1)  # the single-step call ends in a working set and copies back
    ctx.step(st, 4, 2)
    assert_same_bits(by_id(st), one)
    torch.cuda.synchronize()
    ctx.sync_check()
    ctx.close()


@pytest.mark.parametrize("name,n,prec", CASES[:3])
def test_step_captured_in_hip_graph(name, n, prec):
    """rbe_step captured in a HIP graph: every replay (with eager work and
    synchronizations between them) reproduces the direct call bit for bit."""
    p, s = system(name, n=n)
    ctx = rbe.Context(rbe.params_from_preset(p, prec=prec), p["n"])
    st = to_device(s)
    ctx.forces(st, None, None, 0)
    start = snapshot(st)
    ctx.step(st, 3, 1)
    ref = snapshot(st)
    torch.cuda.synchronize()
    ctx.sync_check()
    restore(st, start)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.step(st, 3, 1)
    for rep in range(3):
        restore(st, start)
        junk = torch.randn(4096, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in FIELDS:
            assert torch.equal(getattr(st, k), ref[k]), (rep, k)
        del junk
    ctx.sync_check()
    del g
    ctx.close()


def test_batched_step_split_over_calls_is_bit_identical():
    """The batched form: 1 + 2 + 4 steps equal 7 steps in one call (first
    and last steps launched directly on the caller's arrays, the ones
    between through the two-step graph)."""
    import gen
    from paper_2609_02694_amd import tune
    sizes = [1000, 2400, 5200, 1500]
    reps, cat, off = gen.replica_batch(sizes)
    for prec in (rbe.FP64, rbe.FP32C):
        ctx = rbe.Context.batch(tune.batch_params(reps, 2.5, prec, 2), off)
        st = rbe.Particles.from_numpy(cat)
        ctx.forces(st, None, None, 0)
        start = snapshot(st)
        ctx.step(st, 7, 1)
        one = snapshot(st)
        restore(st, start)
        ctx.step(st, 1, 1)
        ctx.step(st, 2, 2)
        ctx.step(st, 4, 4)
        for k in FIELDS:
            assert torch.equal(getattr(st, k), one[k]), (prec, k)
        torch.cuda.synchronize()
        ctx.sync_check()
        ctx.close()


@pytest.mark.parametrize("name,n,prec,ncell", [
    ("plain3k", None, rbe.FP64, (12, 4, 4)),
    ("electrolyte1m", 20_000, rbe.FP32C, (40, 10, 10)),
    ("subdomain64m", 40_000, rbe.FP32C, (48, 12, 12)),
])
def test_step_returns_cell_order(name, n, prec, ncell):
    """rbe_step returns the particles sorted by the cell keys of their final
    positions (the drift kernels compute those keys): binning the returned
    state again with rbe_build_cells is the identity permutation."""
    p, s = system(name, n=n)
    params = rbe.params_from_preset(p, prec=prec, ncell=ncell)
    ctx = rbe.Context(params, p["n"])
    st = to_device(s)
    ctx.forces(st, None, None, 0)
    for nsteps in (1, 3):
        ctx.step(st, nsteps, 1)
        cs, perm = ctx.build_cells(st.x, st.y, st.z, st.q)
        torch.cuda.synchronize()
        assert torch.equal(perm.cpu(), torch.arange(p["n"], dtype=torch.int32)), nsteps
    ctx.sync_check()
    ctx.close()
