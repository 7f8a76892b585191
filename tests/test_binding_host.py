"""Host-side argument checks of the Python binding (no GPU needed)."""
import pytest

torch = pytest.importorskip("torch")

from paper_2306_09537_amd.quadswarm import QuadSwarm  # noqa: E402


def test_dev_refuses_host_misshaped_and_mistyped_tensors():
    sim = QuadSwarm.__new__(QuadSwarm)  # validation only: no handle is created
    sim._di = 0
    with pytest.raises(ValueError):
        sim._dev(torch.zeros(4, 4), (4, 4))               # host memory
    with pytest.raises(ValueError):
        sim._dev(torch.zeros(4, 4).t(), (4, 4))           # host and not contiguous
    with pytest.raises(ValueError):
        sim._dev(None, (4, 4))                            # not a tensor
    with pytest.raises(ValueError):
        sim._dev(torch.zeros(4, 4, dtype=torch.float64), (4, 4))
