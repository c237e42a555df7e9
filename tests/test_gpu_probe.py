"""The vector-ALU issue-rate probe (measurement support): every mix runs,
times itself and leaves finite values in its output."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_02694_amd as rbe  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rbe.load()


@pytest.mark.parametrize("kind", rbe.PROBE_KINDS)
def test_probe_mix_runs(kind):
    print(f"probe {kind}", flush=True)
    ms = rbe.probe_valu(kind, blocks=64, iters=20)
    assert ms > 0.0
