"""Host-side argument checks of the Python binding (no GPU needed): the
overlap rule of the C ABI and tensor validation."""
import pytest

torch = pytest.importorskip("torch")

from paper_2306_09537_amd.quadswarm import QuadSwarm  # noqa: E402


def test_disjoint_accepts_separate_buffers():
    a, b, c = torch.zeros(8), torch.zeros(8), torch.zeros(4)
    QuadSwarm._disjoint([a, b], [c])
    QuadSwarm._disjoint([a, None], [None, b])


def test_disjoint_refuses_overlaps():
    base = torch.zeros(16)
    with pytest.raises(ValueError):
        QuadSwarm._disjoint([base[:8]], [base[4:12]])   # output overlaps an input
    with pytest.raises(ValueError):
        QuadSwarm._disjoint([base[:8], base[7:9]])      # two outputs overlap
    QuadSwarm._disjoint([base[:8]], [base[8:]])          # adjacent is fine


def test_dev_refuses_host_and_misshaped_tensors():
    sim = QuadSwarm.__new__(QuadSwarm)  # validation only: no handle is created
    sim._di = 0
    with pytest.raises(ValueError):
        sim._dev(torch.zeros(4, 4), (4, 4))               # host memory
    with pytest.raises(ValueError):
        sim._dev(torch.zeros(4, 4).t(), (4, 4))           # not a CUDA tensor either
