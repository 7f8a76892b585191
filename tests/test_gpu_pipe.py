"""Calls of several substeps on small batches of 8-quad swarms run the
motor part one substep ahead in a second wavefront (step_pipe_kernel).
Observation, reward, state, contacts and the device substep counter equal
the one-wavefront kernel's bit for bit, in eager and graph mode."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2306_09537_amd import workloads as W  # noqa: E402
from paper_2306_09537_amd.quadswarm import QuadSwarm  # noqa: E402
from tests.test_gpu_reward import eventful  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def run(w, mode, monkeypatch, nsub, calls, reward, graph=False):
    monkeypatch.setenv("QS_STEP_PIPE", mode)
    sim = QuadSwarm.from_workload(w)
    sim.record_contacts(True)
    if reward:
        sim.set_reward_weights(np.asarray(W.REWARD_WEIGHTS, np.float32))
    g = dev(w.goals)
    outs = []
    if graph:
        sim.set_graph_mode(True)
        buf = dev(w.actions(0))
        obs = torch.empty((w.n_quads, w.obs_dim), device="cuda")
        rew = torch.empty(w.n_quads, device="cuda")
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            if reward:
                sim.step_observe_reward(buf, nsub, g, obs, rew)
            else:
                sim.step_observe(buf, nsub, g, obs)
        for c in range(calls):
            buf.copy_(dev(w.actions(c)))
            gr.replay()
            torch.cuda.synchronize()
            outs.append((obs.clone(), rew.clone() if reward else None))
        t_dev = sim.substep  # the device counter the replays advanced
        sim.set_graph_mode(False)
    else:
        for c in range(calls):
            a = dev(w.actions(c))
            if reward:
                o, r = sim.step_observe_reward(a, nsub, g)
            else:
                o, r = sim.step_observe(a, nsub, g), None
            outs.append((o, r))
    st, t = sim.get_state()
    if graph:
        t = t_dev
    cm = sim.debug_contacts()
    sim.sync()
    res = ([o.cpu() for o, _ in outs], [None if r is None else r.cpu() for _, r in outs],
           st.cpu(), t, cm.cpu())
    sim.close()
    return res


@pytest.mark.parametrize("nsub,reward,flags", [(10, False, W.SWARM_FLAGS),
                                               (2, True, W.SWARM_FLAGS | W.QS_SENSOR_NOISE),
                                               (5, True, W.SWARM_FLAGS | W.QS_DOWNWASH)])
def test_two_wavefront_step_is_bit_identical(nsub, reward, flags, monkeypatch):
    w = eventful(W.custom([8] * 20, seed=41, k=6, flags=flags, name="swarm8"), 9)
    a = run(w, "0", monkeypatch, nsub, 6, reward)
    b = run(w, "1", monkeypatch, nsub, 6, reward)
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)
    if reward:
        for x, y in zip(a[1], b[1]):
            assert torch.equal(x, y)
    assert torch.equal(a[2], b[2]) and a[3] == b[3] == 6 * nsub
    assert torch.equal(a[4], b[4])


def test_two_wavefront_step_graph_replays(monkeypatch):
    w = eventful(W.custom([8] * 24, seed=42, k=6, flags=W.SWARM_FLAGS | W.QS_SENSOR_NOISE,
                          name="swarm8"), 10)
    a = run(w, "0", monkeypatch, 4, 3, True, graph=True)
    b = run(w, "1", monkeypatch, 4, 3, True, graph=True)
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        assert torch.equal(x, y)
    assert torch.equal(a[2], b[2]) and a[3] == b[3] == 12
