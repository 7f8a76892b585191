"""Full-size parity in the launch configurations the benchmark times, on
sampled environments the oracle can follow one by one:

- 16384 uneven environments (172,943 quads): autotuned persistent bucketed
  launch, one 10-substep call captured as a graph and replayed;
- 32768 x 32 (1,048,576 quads): one-substep and 10-substep launches, and
  the differentiable rollout (100 substeps, checkpoint every 20 calls);
- 1,048,576 x 1: one-substep and 10-substep launches;
- 2^26 single-quad swarms, the library's quad limit: one launch.

Teacher-forced as in the other parity tests (the oracle restarts from the
GPU's float32 state of the sampled environments after every call); bounds
as there: 1e-5 per substep, 10 x that for 10-substep calls.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2306_09537_amd import workloads as W  # noqa: E402
from paper_2306_09537_amd.quadswarm import QuadSwarm  # noqa: E402
from tests import gpu_util as U  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_uneven_full_size_graph_replay_sampled():
    w = W.uneven(seed=7)
    nsub, reps = 10, 3
    sim = QuadSwarm.from_workload(w)
    g = dev(w.goals)
    out = torch.empty((w.n_quads, w.obs_dim), device="cuda")
    choice = sim.autotune(dev(w.actions(99)), nsub, g, out)
    assert choice["bucketed"]
    buf = torch.empty((w.n_quads, 4), device="cuda")
    obs = torch.empty((w.n_quads, w.obs_dim), device="cuda")
    sim.set_graph_mode(True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        buf.copy_(dev(w.actions(0)))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sim.step_observe(buf, nsub, g, obs)
    fmax = U.fmax_of(w.params)
    samples = [(100, 160), (8000, 8060), (16324, 16384)]
    orcs = [O.Oracle.from_workload(w, e0, e1) for e0, e1 in samples]
    spans = [(int(w.env_offsets[e0]), int(w.env_offsets[e1])) for e0, e1 in samples]
    prev = w.state0.astype(np.float64)
    worst, excluded = 0.0, 0
    for r in range(reps):
        a = w.actions(r)
        buf.copy_(dev(a))
        graph.replay()
        st, _ = sim.get_state()
        torch.cuda.synchronize()
        s_gpu = st.cpu().numpy().astype(np.float64)
        o_gpu = obs.cpu().numpy()
        for orc, (q0, q1), (e0, e1) in zip(orcs, spans, samples):
            ref, _, _, mg = orc.step(prev[q0:q1], a[q0:q1], nsub, r * nsub, margins=True)
            err = U.rel_err(s_gpu[q0:q1], ref, fmax[q0:q1]).max(axis=1)
            near = mg < U.MARGIN
            assert ((err <= 10 * U.TOL) | near).all(), (r, e0)
            excluded += int(near.sum())
            worst = max(worst, float(err[~near].max()))
            o_ref, _ = orc.observe(s_gpu[q0:q1], w.goals[q0:q1].astype(np.float64))
            offs = (w.env_offsets[e0:e1 + 1] - q0).astype(np.int64)
            U.check_obs(o_gpu[q0:q1], o_ref, s_gpu[q0:q1], offs, w.k_neighbors)
        prev = s_gpu
    sim.set_graph_mode(False)
    sim.sync()
    print("uneven full size graph replay: worst", worst, "excluded", excluded, "launch", choice)
    assert worst <= 10 * U.TOL


def sampled_teacher_forced(w, calls, nsub, samples, tol):
    """One handle at full size, qs_step_observe calls of nsub substeps; after
    every call the sampled environment ranges are checked against the
    oracle restarted from the GPU's state (state, contacts, observation)."""
    sim = QuadSwarm.from_workload(w)
    record = bool(w.flags & W.QS_COLLIDE)
    sim.record_contacts(record)
    g = dev(w.goals)
    fmax = U.fmax_of(w.params)
    orcs = [O.Oracle.from_workload(w, e0, e1) for e0, e1 in samples]
    spans = [(int(w.env_offsets[e0]), int(w.env_offsets[e1])) for e0, e1 in samples]
    prev = w.state0
    worst = 0.0
    for call in range(calls):
        a = w.actions(call)
        obs = sim.step_observe(dev(a), nsub, g)
        st, _ = sim.get_state()
        cm = sim.debug_contacts() if record else None
        sim.sync()
        s_gpu = st.cpu().numpy().astype(np.float64)
        o_gpu = obs.cpu().numpy()
        c_gpu = cm.cpu().numpy().view(np.uint64) if record else None
        for orc, (q0, q1), (e0, e1) in zip(orcs, spans, samples):
            ref, c_ref, _, mg = orc.step(prev[q0:q1].astype(np.float64), a[q0:q1], nsub,
                                         call * nsub, margins=True)
            err = U.rel_err(s_gpu[q0:q1], ref, fmax[q0:q1]).max(axis=1)
            near = mg < U.MARGIN
            assert ((err <= tol) | near).all(), (call, e0)
            if (~near).any():
                worst = max(worst, float(err[~near].max()))
            offs = (w.env_offsets[e0:e1 + 1] - q0).astype(np.int64)
            if record and not near.any():
                U.check_contacts(c_gpu[q0:q1], c_ref, s_gpu[q0:q1, 0:3], ref[:, 0:3], offs,
                                 w.consts["col_dist"])
            o_ref, _ = orc.observe(s_gpu[q0:q1], w.goals[q0:q1].astype(np.float64))
            U.check_obs(o_gpu[q0:q1], o_ref, s_gpu[q0:q1], offs, w.k_neighbors)
        prev = s_gpu
    sim.close()
    return worst


@pytest.mark.parametrize("nsub,calls", [(1, 5), (10, 2)])
def test_scale32_full_size_sampled(nsub, calls):
    w = W.scale32(seed=3)
    worst = sampled_teacher_forced(w, calls, nsub, [(0, 16), (20000, 20016), (32752, 32768)],
                                   U.TOL * nsub)
    print("scale32 full size", nsub, "worst", worst)
    assert worst <= U.TOL * nsub


@pytest.mark.parametrize("nsub,calls", [(1, 5), (10, 2)])
def test_scale1_full_size_sampled(nsub, calls):
    w = W.scale1(seed=4)
    worst = sampled_teacher_forced(w, calls, nsub,
                                   [(0, 2048), (524288, 526336), (1046528, 1048576)],
                                   U.TOL * nsub)
    print("scale1 full size", nsub, "worst", worst)
    assert worst <= U.TOL * nsub


def test_large_grid_ragged_tail_sampled():
    """More than 2048 workgroups, so the observation rows leave in several
    staging passes per workgroup, with a partly filled last workgroup:
    16,390 swarms of 8 (2049 workgroups of 64 quads, 48 in the last).
    Sampled at the start, the middle and the last swarms."""
    w = W.custom([8] * 16390, seed=11, k=6, name="ragged_16390x8")
    assert w.n_quads % 64 == 48
    worst = sampled_teacher_forced(w, 3, 1, [(0, 8), (8000, 8016), (16374, 16390)], U.TOL)
    print("ragged large grid worst", worst)
    assert worst <= U.TOL


def test_maximum_size_sampled():
    """The largest handle the library takes: 2^26 single-quad swarms (its
    quad limit), 64 tiles of the 1,048,576 x 1 workload's parameters and
    states (each tile draws its own noise: the noise is keyed by the global
    quad index).  One step + observation, sampled at the start, the middle
    and the end of the quad range."""
    base = W.scale1(seed=5)
    reps = 64
    q = base.n_quads * reps
    assert q == 1 << 26
    w = base.with_(env_sizes=np.ones(q, np.int32), env_offsets=np.arange(q + 1, dtype=np.int32),
                   params=np.tile(base.params, (reps, 1)), state0=np.tile(base.state0, (reps, 1)),
                   goals=np.tile(base.goals, (reps, 1)))
    worst = sampled_teacher_forced(w, 1, 1, [(0, 2048), (q // 2 - 1024, q // 2 + 1024),
                                             (q - 2048, q)], U.TOL)
    print("maximum size worst", worst)
    assert worst <= U.TOL


def test_scale32_fwd_bwd_full_size_sampled():
    """The benchmark's 32768 x 32 differentiable rollout (100 substeps,
    checkpoint every 20 calls, penalty on): gradients of envs 5000 and
    5001 against the oracle's reverse mode, block by block with the
    oracle-derived bounds of the other gradient tests."""
    from tests.test_gpu_grad import check, gpu_grads, oracle_grads, oracle_pert
    w = W.scale32(seed=0)
    T, nsub, ce = 100, 1, 20
    acts = w.action_sequence(T)
    rng = np.random.default_rng(5)
    Wt = rng.normal(size=(w.n_quads, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = rng.uniform(0.5, 2.0, size=w.n_quads).astype(np.float32)
    gs, gact, gpar, *_ = gpu_grads(w, acts, nsub, Wt, gpen, ce)
    assert np.isfinite(gs).all() and np.isfinite(gact).all() and np.isfinite(gpar).all()
    e0, e1 = 5000, 5002
    q0, q1 = int(w.env_offsets[e0]), int(w.env_offsets[e1])
    g_ref = oracle_grads(w, acts, nsub, Wt, gpen, env_range=(e0, e1))
    g_pert = oracle_pert(w, acts, nsub, Wt, gpen, 5, env_range=(e0, e1))
    check((gs[q0:q1], gact[:, q0:q1], gpar[q0:q1]), g_ref, g_pert, "32768 x 32 sampled")


def test_diff_fwd_bwd_full_size_sampled():
    """The benchmark's 1024 x 8 differentiable rollout in its launch
    configuration (200 substeps, checkpoint every 20 calls, penalty on:
    the three-wavefront forward, the two-wavefront recompute and the
    four-wavefront reverse sweep): gradients of the first two, two middle
    and the last two environments against the oracle's reverse mode, block
    by block with the oracle-derived bounds of the other gradient tests."""
    from tests.test_gpu_grad import check, gpu_grads, oracle_grads, oracle_pert
    w = W.diff(seed=0)
    T, nsub, ce = 200, 1, 20
    acts = w.action_sequence(T)
    rng = np.random.default_rng(6)
    Wt = rng.normal(size=(w.n_quads, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = rng.uniform(0.5, 2.0, size=w.n_quads).astype(np.float32)
    gs, gact, gpar, *_ = gpu_grads(w, acts, nsub, Wt, gpen, ce)
    assert np.isfinite(gs).all() and np.isfinite(gact).all() and np.isfinite(gpar).all()
    for e0, e1 in ((0, 2), (511, 513), (1022, 1024)):
        q0, q1 = int(w.env_offsets[e0]), int(w.env_offsets[e1])
        g_ref = oracle_grads(w, acts, nsub, Wt, gpen, env_range=(e0, e1))
        g_pert = oracle_pert(w, acts, nsub, Wt, gpen, 5, env_range=(e0, e1))
        check((gs[q0:q1], gact[:, q0:q1], gpar[q0:q1]), g_ref, g_pert,
              f"1024 x 8 envs {e0}-{e1}")
