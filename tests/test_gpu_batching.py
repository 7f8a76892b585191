"""Uneven-size batching on the GPU: the persistent bucketed launch, graph
capture of rollouts with a device-side substep counter, and the autotuner.

The bucketed launch changes only which lanes serve which quads, not the
arithmetic of any quad, so its results must equal the one-workgroup-per-
block table path bit for bit; both are also checked against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2306_09537_amd import workloads as W  # noqa: E402
from paper_2306_09537_amd.quadswarm import QuadSwarm  # noqa: E402
from tests.test_gpu_parity import teacher_forced  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def run_calls(sim, w, calls, nsub):
    g = dev(w.goals)
    sim.record_contacts(True)
    outs = []
    for c in range(calls):
        o = sim.step_observe(dev(w.actions(c)), nsub, g)
        outs.append((o.clone(), sim.get_state()[0].clone(), sim.debug_contacts().clone()))
    sim.sync()
    return outs


def mixed_sizes(seed, n_envs):
    """Every size 1..64, including non-powers of two (padded slots)."""
    rng = np.random.default_rng(seed)
    return list(rng.integers(1, 65, size=n_envs)) + list(range(1, 65))


@pytest.mark.parametrize("k", [6, 0, 3])
def test_bucketed_equals_table_path_bitwise(k, monkeypatch):
    w = W.custom(mixed_sizes(1, 150), seed=1, k=k, name="mixed")
    monkeypatch.setenv("QS_BUCKETED", "0")
    a = run_calls(QuadSwarm.from_workload(w), w, 6, 5)
    monkeypatch.setenv("QS_BUCKETED", "1")
    b = run_calls(QuadSwarm.from_workload(w), w, 6, 5)
    for (oa, sa, ca), (ob, sb, cb) in zip(a, b):
        assert torch.equal(sa, sb)
        assert torch.equal(oa, ob)
        assert torch.equal(ca, cb)


@pytest.mark.parametrize("k,obs", [(6, True), (6, False), (3, True), (0, True)])
def test_chunked_partner_bodies_equal_table_path_bitwise(k, obs, monkeypatch):
    """Slots of 16 and 32 with the chunked partner body: results equal the
    table path bit for bit, in eager calls and replays of a captured graph."""
    w = W.custom(mixed_sizes(3, 150), seed=3, k=k, name="mixed")
    monkeypatch.setenv("QS_BUCKETED", "0")
    ref = QuadSwarm.from_workload(w)
    monkeypatch.setenv("QS_BUCKETED", "1")
    sim = QuadSwarm.from_workload(w)
    sim.set_partner_chunks([16, 32])
    plan = sim.launch_plan()
    assert [r["slot"] for r in plan] == [64, 32, 16, 8, 4, 2, 1]
    assert [r["chunked"] for r in plan] == [False, True, True, False, False, False, False]
    assert sum(r["swarms"] for r in plan) == w.n_envs
    g = dev(w.goals)
    for c in range(5):
        a = dev(w.actions(c))
        if obs:
            assert torch.equal(sim.step_observe(a, 4, g), ref.step_observe(a, 4, g))
        else:
            sim.step(a, 4)
            ref.step(a, 4)
    assert torch.equal(sim.get_state()[0], ref.get_state()[0])
    # graph mode
    nsub, calls = 3, 3
    acts = torch.stack([dev(w.actions(10 + c)) for c in range(calls)])
    out = torch.empty((calls, w.n_quads, w.obs_dim), device="cuda")
    sim.set_graph_mode(True)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for c in range(calls):
            sim.step_observe(acts[c], nsub, g, out[c])
    for r in range(2):
        graph.replay()
        torch.cuda.synchronize()
        for c in range(calls):
            assert torch.equal(out[c], ref.step_observe(acts[c], nsub, g)), f"replay {r} call {c}"
    sim.set_graph_mode(False)
    sim.sync()


def test_autotune_per_slot_table():
    """The autotuner times the items of slots 16 and 32 alone with each
    partner body and keeps the chunked one only where it was faster; the
    table lists every slot size with its swarm count."""
    w = W.uneven(seed=9, n_envs=4096)
    sim = QuadSwarm.from_workload(w)
    g = dev(w.goals)
    out = torch.empty((w.n_quads, w.obs_dim), device="cuda")
    choice = sim.autotune(dev(w.actions(0)), 10, g, out)
    print("autotune", choice)
    sizes, counts = np.unique(w.env_sizes, return_counts=True)
    slots = {r["slot"]: r for r in choice["slots"]}
    assert set(slots) == set(int(x) for x in sizes)
    for n, cnt in zip(sizes, counts):
        assert slots[int(n)]["swarms"] == cnt
    for n in (16, 32):
        r = slots[n]
        assert r["ns_one"] > 0 and r["ns_chunked"] > 0
        if r["chunked"]:
            assert r["ns_chunked"] < r["ns_one"]
    for n in (1, 2, 4, 8):
        assert not slots[n]["chunked"] and slots[n]["ns_one"] == 0
    sim.sync()


def test_bucketed_uneven_parity_with_oracle():
    w = W.uneven(seed=3, n_envs=400)
    st = teacher_forced(w, 60)
    assert st["contacts"] > 0
    w2 = W.custom(mixed_sizes(2, 60), seed=2, k=6, name="mixed")
    st2 = teacher_forced(w2, 40)
    assert st2["max_err"] <= 1e-5 and st["max_err"] <= 1e-5


@pytest.mark.parametrize("workload", ["uneven", "swarm8"])
def test_graph_replay_matches_eager(workload):
    """Capture 10 calls of qs_step_observe (10 substeps each) in graph mode;
    replay 3 times with new actions copied in between and eager work of the
    program in between; every replay equals the eager run of the same calls
    (noise counters advance on the device)."""
    w = (W.uneven(seed=4, n_envs=512) if workload == "uneven" else W.swarm8(seed=4, n_envs=256))
    nsub, calls, reps = 10, 10, 3
    g = dev(w.goals)
    acts_all = [dev(w.actions(c)) for c in range(calls * reps)]
    buf = torch.empty((calls, w.n_quads, 4), device="cuda")
    obs = torch.empty((calls, w.n_quads, w.obs_dim), device="cuda")
    sim = QuadSwarm.from_workload(w)
    sim.set_graph_mode(True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm up the stream outside capture
        buf.copy_(torch.stack(acts_all[:calls]))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for c in range(calls):
            sim.step_observe(buf[c], nsub, g, obs[c])
    # capture records launches without running them: state and counter untouched
    assert sim.substep == 0
    ref = QuadSwarm.from_workload(w)
    for r in range(reps):
        buf.copy_(torch.stack(acts_all[r * calls:(r + 1) * calls]))
        graph.replay()
        torch.cuda.synchronize()
        ref_obs = []
        for c in range(calls):
            ref_obs.append(ref.step_observe(acts_all[r * calls + c], nsub, g).clone())
        ref_state, _ = ref.get_state()
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work
        got_state, _ = sim.get_state()
        torch.cuda.synchronize()
        assert sim.substep == (r + 1) * calls * nsub
        assert torch.equal(got_state, ref_state), f"replay {r}"
        for c in range(calls):
            assert torch.equal(obs[c], ref_obs[c]), f"replay {r} call {c}"
    sim.set_graph_mode(False)
    assert sim.substep == reps * calls * nsub
    sim.sync()


@pytest.mark.parametrize("workload", ["uneven", "swarm8"])
def test_autotune_keeps_state_and_results(workload):
    w = (W.uneven(seed=5, n_envs=1024) if workload == "uneven" else W.swarm8(seed=5, n_envs=2048))
    g = dev(w.goals)
    a = QuadSwarm.from_workload(w)
    b = QuadSwarm.from_workload(w)
    for c in range(3):
        a.step(dev(w.actions(c)), 2)
        b.step(dev(w.actions(c)), 2)
    before, t0 = a.get_state()
    before = before.clone()
    out = torch.empty((w.n_quads, w.obs_dim), device="cuda")
    choice = a.autotune(dev(w.actions(99)), 10, g, out)
    after, t1 = a.get_state()
    torch.cuda.synchronize()
    print("autotune", workload, choice)
    assert choice["block"] in (64, 128)
    assert choice["bucketed"] == (workload == "uneven")
    assert t0 == t1 and torch.equal(before, after)
    for c in range(3, 6):
        oa = a.step_observe(dev(w.actions(c)), 10, g)
        ob = b.step_observe(dev(w.actions(c)), 10, g)
        assert torch.equal(oa, ob)
    assert torch.equal(a.get_state()[0], b.get_state()[0])
    a.sync()


# ------------------------------------------------------------------ downwash
def stacked_swarms(seed, n_envs=64, n=8, noise=False):
    """Swarms stacked in narrow columns so that downwash is frequent."""
    c = dict(dw_noise_a=0.3, dw_noise_w=2.0) if noise else {}
    w = W.custom([n] * n_envs, seed=seed, k=6, flags=W.SWARM_FLAGS | W.QS_DOWNWASH,
                 name="stacked", **c)
    rng = np.random.default_rng(seed)
    s0 = w.state0.copy()
    for e in range(n_envs):
        base = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), 2.0])
        for i in range(n):
            s0[e * n + i, 0:3] = base + [rng.normal(0, 0.04), rng.normal(0, 0.04), 0.22 * i]
    return w.with_(state0=s0.astype(np.float32))


@pytest.mark.parametrize("noise", [False, True])
def test_downwash_parity_with_oracle(noise):
    from oracle import oracle as O
    w = stacked_swarms(6, noise=noise)
    st = teacher_forced(w, 80)
    assert st["max_err"] <= 1e-5
    # downwash really acted
    orc = O.Oracle.from_workload(w)
    _, _, ev = orc.step(w.state0.astype(np.float64), w.actions(0), 1, 0)
    assert np.count_nonzero(ev & O.EV_DOWNWASH) > 50


def test_downwash_bucketed_equals_table_and_rollout_equals_steps(monkeypatch):
    w = stacked_swarms(7, n_envs=40).with_(
        env_sizes=np.array([8] * 40, np.int32))
    sizes = [8, 3, 5, 8, 2, 7] * 6 + [8] * 4
    w2 = W.custom(sizes, seed=7, k=6, flags=W.SWARM_FLAGS | W.QS_DOWNWASH, name="mixed-dw")
    s0 = w2.state0.copy()
    rng = np.random.default_rng(7)
    q = 0
    for n in sizes:
        base = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), 2.0])
        for i in range(n):
            s0[q, 0:3] = base + [rng.normal(0, 0.04), rng.normal(0, 0.04), 0.22 * i]
            q += 1
    w2 = w2.with_(state0=s0.astype(np.float32))
    monkeypatch.setenv("QS_BUCKETED", "0")
    a = run_calls(QuadSwarm.from_workload(w2), w2, 5, 4)
    monkeypatch.setenv("QS_BUCKETED", "1")
    b = run_calls(QuadSwarm.from_workload(w2), w2, 5, 4)
    for (oa, sa, ca), (ob, sb, cb) in zip(a, b):
        assert torch.equal(sa, sb) and torch.equal(oa, ob) and torch.equal(ca, cb)
    sim = QuadSwarm.from_workload(w)
    ref = QuadSwarm.from_workload(w)
    acts = np.stack([w.actions(c) for c in range(6)])
    sim.rollout(dev(acts), 3)
    for c in range(6):
        ref.step(dev(acts[c]), 3)
    assert torch.equal(sim.get_state()[0], ref.get_state()[0])
    from paper_2306_09537_amd.quadswarm import QuadSwarmError
    gs = torch.zeros((w.n_quads, 27), device="cuda")
    with pytest.raises(QuadSwarmError) as ei:
        sim.step_backward(sim.get_state()[0], dev(acts[0]), 1, 0, gs, gs.clone(),
                          torch.zeros((w.n_quads, 4), device="cuda"),
                          torch.zeros((w.n_quads, 6), device="cuda"))
    assert ei.value.code == -8
