"""GPU test of qs_step_backward_noalloc, the allocation-free form of
qs_step_backward (fixed per-device scratch), through the C ABI: its outputs
equal those of qs_step_backward bit for bit on two calls in a row, the
second with a smaller input (fewer quads, fewer substeps), and a request
beyond the fixed scratch is refused with QS_ERR_TOO_LARGE."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2306_09537_amd import workloads as W  # noqa: E402
from paper_2306_09537_amd.quadswarm import QuadSwarm, QuadSwarmError  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def both(sim, w, nsub, seed):
    """(qs_step_backward outputs, qs_step_backward_noalloc outputs) of one
    call from the handle's current state."""
    rng = np.random.default_rng(seed)
    Q = w.n_quads
    s_in, t = sim.get_state()
    act = dev(w.actions(seed))
    gout = dev(rng.normal(size=(Q, 27)))
    gpar0 = dev(rng.normal(size=(Q, 6)))  # the parameter gradient is added to it
    outs = []
    for fn in (sim.step_backward, sim.step_backward_noalloc):
        gin = torch.full((Q, 27), np.nan, device="cuda")
        gact = torch.full((Q, 4), np.nan, device="cuda")
        gpar = gpar0.clone()
        fn(s_in, act, nsub, t, gout, gin, gact, gpar)
        torch.cuda.synchronize()
        outs.append((gin.cpu(), gact.cpu(), gpar.cpu()))
    sim.sync()
    return outs


@pytest.mark.parametrize("first,second", [((W.swarm8, 512, 3), (W.swarm8, 64, 1)),
                                          ((W.diff, 1024, 2), ("mixed", 0, 1))])
def test_noalloc_step_backward_equals_step_backward(first, second):
    sims = []
    for k, (mk, n_envs, nsub) in enumerate((first, second)):
        if mk == "mixed":
            w = W.custom([8, 3, 5, 2, 7, 16, 1, 4] * 10, seed=60, k=6, name="mixed")
        else:
            w = mk(seed=k, n_envs=n_envs)
        sim = QuadSwarm.from_workload(w)
        sim.step(dev(w.actions(100)), 2)  # a state off the initial one
        ref, got = both(sim, w, nsub, 7 + k)
        for r, g in zip(ref, got):
            assert torch.isfinite(r).all()
            assert torch.equal(r, g)
        sims.append(sim)
    # the second call had the smaller input
    assert sims[1].n_quads < sims[0].n_quads
    for sim in sims:
        sim.close()


def test_noalloc_refuses_requests_beyond_its_scratch():
    """(60 + 31 n_substeps) Q floats must fit 64 MiB: 150,000 quads fit one
    substep and are refused with two, before anything is enqueued."""
    w = W.custom([1] * 150000, seed=61, k=0, flags=W.QS_FLOOR, name="big")
    sim = QuadSwarm.from_workload(w)
    Q = w.n_quads
    s_in, t = sim.get_state()
    act = dev(w.actions(0))
    gout = torch.zeros((Q, 27), device="cuda")
    gin = torch.zeros((Q, 27), device="cuda")
    gact = torch.zeros((Q, 4), device="cuda")
    gpar = torch.zeros((Q, 6), device="cuda")
    sim.step_backward_noalloc(s_in, act, 1, t, gout, gin, gact, gpar)
    with pytest.raises(QuadSwarmError) as ei:
        sim.step_backward_noalloc(s_in, act, 2, t, gout, gin, gact, gpar)
    assert ei.value.code == -9
    sim.sync()
    sim.close()
