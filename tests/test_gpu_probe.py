"""The claim-latency probe: the time of one dependent returning atomic, the
latency the step loop's steps wait on at least once each."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ibip = pytest.importorskip("paper_2101_03240_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_probe_claim_latency(dev):
    l2 = ibip.probe_claim_latency(256 << 10, 2000, device=dev)
    far = ibip.probe_claim_latency(256 << 20, 2000, device=dev)
    assert 0 < l2 < 1e5 and 0 < far < 1e5


def test_probe_rejects_bad_spans(dev):
    with pytest.raises(ibip.IbipError):
        ibip.probe_claim_latency(1024, 10, device=dev)
    with pytest.raises(ibip.IbipError):
        ibip.probe_claim_latency(1 << 34, 10, device=dev)
    with pytest.raises(ibip.IbipError):
        ibip.probe_claim_latency(1 << 20, 0, device=dev)
