"""GPU differentiation parity: the HIP rollout and adjoint kernels (through
the C ABI) against the FP64 oracle's reverse-mode derivative, which the CPU
tests pin to central differences.

Tolerance: the GPU integrates and differentiates in float32, so its
trajectory drifts from the float64 one by the chaos of the tumbling swarm.
The comparison is block by block (tests/grad_check.py): each state field
group, each rotor's action gradient and each parameter column on its own
scale, norm-wise and element-wise, against bounds derived from the oracle
itself (10 x the change of the oracle's own gradient when its initial state
is perturbed by 2^-23 relative noise, with floors 1e-4 and 2e-4).  A norm
over all parameters at once would not see the thrust-to-weight or tau_m
columns, which carry ~1e-5 of it on a dense swarm.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2306_09537_amd import workloads as W  # noqa: E402
from paper_2306_09537_amd.quadswarm import QuadSwarm, rollout  # noqa: E402
from tests import grad_check as G  # noqa: E402
from tests.test_oracle_grad import LOSSY, dense_problem  # noqa: E402

pytestmark = pytest.mark.gpu
BETA = 100.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def problem(seed, T, n_envs=4, **kw):
    w, s0 = dense_problem(seed, n_envs=n_envs, **kw)
    w = w.with_(state0=s0.astype(np.float32))
    rng = np.random.default_rng(seed + 100)
    acts = rng.uniform(0.05, 0.95, size=(T, w.n_quads, 4)).astype(np.float32)
    Wt = rng.normal(size=(w.n_quads, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = rng.uniform(0.5, 2.0, size=w.n_quads).astype(np.float32)
    return w, acts, Wt, gpen


def oracle_grads(w, acts, nsub, Wt, gpen, s0=None, env_range=None):
    orc = O.Oracle.from_workload(w, *(env_range or (0, w.n_envs)))
    q0 = int(w.env_offsets[env_range[0]]) if env_range else 0
    q1 = int(w.env_offsets[env_range[1]]) if env_range else w.n_quads
    s = (w.state0 if s0 is None else s0)[q0:q1].astype(np.float64)
    gp = None if gpen is None else gpen[q0:q1].astype(np.float64)
    return orc.rollout_vjp(s, acts[:, q0:q1].astype(np.float64), nsub, 0,
                           Wt[q0:q1].astype(np.float64), gp, None if gpen is None else BETA)


def oracle_pert(w, acts, nsub, Wt, gpen, seed=0, env_range=None):
    """The oracle's gradient from an initial state perturbed by 2^-23
    relative noise (the size of one float32 rounding)."""
    rng = np.random.default_rng(seed)
    s0 = w.state0.astype(np.float64)
    s0p = s0 * (1 + rng.uniform(-1, 1, size=s0.shape) * 2.0 ** -23)
    return oracle_grads(w, acts, nsub, Wt, gpen, s0=s0p, env_range=env_range)


def check(got, ref, pert, title):
    """Every block of the GPU gradient against the oracle's (see grad_check)."""
    rows = G.compare(got, ref, pert)
    print(G.report(rows, title))
    assert not G.failures(rows), G.report(G.failures(rows), title + " failures")
    return rows


def gpu_grads(w, acts, nsub, Wt, gpen, ce):
    sim = QuadSwarm.from_workload(w)
    T = acts.shape[0]
    a = dev(acts)
    n_ck = (T + ce - 1) // ce
    ckpt = torch.empty((n_ck, 27, w.n_quads), device="cuda")
    pen = torch.zeros(w.n_quads, device="cuda")
    sim.rollout(a, nsub, ce, ckpt, pen, BETA)
    sT, tT = sim.get_state()
    gs = dev(Wt).clone()
    gact = torch.empty_like(a)
    gpar = torch.zeros((w.n_quads, 6), device="cuda")
    sim.rollout_backward(a, nsub, ce, ckpt, 0, gs, None if gpen is None else dev(gpen), BETA,
                         gact, gpar)
    sim.sync()
    out = (gs.cpu().numpy(), gact.cpu().numpy(), gpar.cpu().numpy(), sT.cpu().numpy(),
           pen.cpu().numpy(), ckpt.cpu().numpy(), tT)
    sim.close()
    return out


@pytest.mark.parametrize("n", [8, 32])
def test_rollout_forward_matches_steps_and_oracle_penalty(n):
    """The differentiable rollout (penalty on) reaches the state of repeated
    steps bit for bit, checkpoints included, and the oracle's penalty; in
    swarms of 32 the two take different routes to the same contact sets
    (the rollout's pass over every partner, the steps' screen and exact
    test)."""
    w, acts, Wt, gpen = problem(0, 24, n=n)
    T, nsub, ce = 24, 2, 5
    sim = QuadSwarm.from_workload(w)
    ckpt = torch.empty((5, 27, w.n_quads), device="cuda")
    pen = torch.zeros(w.n_quads, device="cuda")
    sim.rollout(dev(acts), nsub, ce, ckpt, pen, BETA)
    sT, t = sim.get_state()
    ref = QuadSwarm.from_workload(w)
    cks = []
    for c in range(T):
        if c % ce == 0:
            cks.append(ref.get_state()[0].clone())
        ref.step(dev(acts[c]), nsub)
    sR, _ = ref.get_state()
    torch.cuda.synchronize()
    assert t == T * nsub
    assert torch.equal(sT, sR)
    for k, s in enumerate(cks):
        assert torch.equal(ckpt[k].T.contiguous(), s)
    _, pen_o = O.Oracle.from_workload(w).rollout(w.state0.astype(np.float64),
                                                 acts.astype(np.float64), nsub, 0, beta=BETA)
    assert pen_o.max() > 1e-3
    np.testing.assert_allclose(pen.cpu().numpy(), pen_o, rtol=2e-4, atol=1e-7)


@pytest.mark.parametrize("seed,T,nsub,ce,c", [(0, 30, 2, 7, {}), (1, 60, 1, 20, {}), (3, 20, 5, 3, {}),
                                              (2, 30, 2, 7, LOSSY)])
def test_adjoint_matches_oracle(seed, T, nsub, ce, c):
    w, acts, Wt, gpen = problem(seed, T, **c)
    g_ref = oracle_grads(w, acts, nsub, Wt, gpen)
    g_pert = oracle_pert(w, acts, nsub, Wt, gpen, seed)
    gs, gact, gpar, *_ = gpu_grads(w, acts, nsub, Wt, gpen, ce)
    got = (gs, gact, gpar)
    check(got, g_ref, g_pert, f"adjoint seed {seed}")
    # the check sees a wrong small column: each of these, zeroed in a copy of
    # the GPU's gradient, fails it (and nothing else does)
    for blk in ("param.t2w", "param.tau_m", "param.mass"):
        failed = [r[0] for r in G.failures(G.compare(G.zeroed(got, blk), g_ref, g_pert))]
        assert failed == [blk], (blk, failed)


@pytest.mark.parametrize("block", ["64", "128"])
def test_adjoint_large_swarms_match_oracle(block, monkeypatch):
    """Swarms of 32 (in-swarm loops at run time in the differentiation
    kernels), in workgroups of one and of two wavefronts (the latter with
    workgroup barriers): penalty and gradients against the oracle."""
    monkeypatch.setenv("QS_BLOCK_SIZE", block)
    w, acts, Wt, gpen = problem(6, 16, n_envs=5, n=32, spread=0.6)
    nsub, ce = 1, 5
    g_ref = oracle_grads(w, acts, nsub, Wt, gpen)
    g_pert = oracle_pert(w, acts, nsub, Wt, gpen, 6)
    gs, gact, gpar, sT, pen, *_ = gpu_grads(w, acts, nsub, Wt, gpen, ce)
    _, pen_o = O.Oracle.from_workload(w).rollout(w.state0.astype(np.float64),
                                                 acts.astype(np.float64), nsub, 0, beta=BETA)
    assert pen_o.max() > 1e-3
    np.testing.assert_allclose(pen, pen_o, rtol=2e-4, atol=1e-7)
    check((gs, gact, gpar), g_ref, g_pert, f"n = 32 adjoint, block {block}")


def sized_problem(seed, T, sizes, spread=0.3, z=3.0):
    """Swarms of the given sizes packed within +-spread m of a centre each
    (contacts and penalty active), actions U(0.05, 0.95)."""
    w = W.custom(list(sizes), seed=seed, k=6, flags=W.SWARM_FLAGS, name="sized")
    rng = np.random.default_rng(seed)
    s0 = w.state0.astype(np.float64).copy()
    for e in range(w.n_envs):
        q0, q1 = int(w.env_offsets[e]), int(w.env_offsets[e + 1])
        s0[q0:q1, 0:3] = rng.uniform(-2, 2, 3) * [1, 1, 0] + [0, 0, z] + \
            rng.uniform(-spread, spread, size=(q1 - q0, 3))
    w = w.with_(state0=s0.astype(np.float32))
    rng = np.random.default_rng(seed + 100)
    acts = rng.uniform(0.05, 0.95, size=(T, w.n_quads, 4)).astype(np.float32)
    Wt = rng.normal(size=(w.n_quads, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = rng.uniform(0.5, 2.0, size=w.n_quads).astype(np.float32)
    return w, acts, Wt, gpen


@pytest.mark.parametrize("sizes,pen", [([8, 3, 5, 2, 7, 16] * 3, True),
                                       ([8, 3, 5, 2, 7, 16] * 3, False),
                                       ([4] * 24, True), ([16] * 6, True), ([16] * 6, False)])
def test_table_path_adjoint_matches_oracle(sizes, pen):
    """Uneven swarm sizes and uniform sizes other than 1, 8 and 32 run the
    table-mapped rollout, recompute and reverse kernels (run-time swarm
    sizes from the host-built table); with and without the penalty, block by
    block against the oracle's derivative."""
    w, acts, Wt, gpen = sized_problem(40 + len(sizes), 16, sizes)
    if not pen:
        gpen = None
    nsub, ce = 2, 5
    g_ref = oracle_grads(w, acts, nsub, Wt, gpen)
    g_pert = oracle_pert(w, acts, nsub, Wt, gpen, 40)
    gs, gact, gpar, sT, pen_g, *_ = gpu_grads(w, acts, nsub, Wt, gpen, ce)
    _, pen_o = O.Oracle.from_workload(w).rollout(w.state0.astype(np.float64),
                                                 acts.astype(np.float64), nsub, 0, beta=BETA)
    assert pen_o.max() > 1e-3
    np.testing.assert_allclose(pen_g, pen_o, rtol=2e-4, atol=1e-7)
    check((gs, gact, gpar), g_ref, g_pert, f"table path sizes {sorted(set(sizes))} pen {pen}")


@pytest.mark.parametrize("n,pen", [(8, True), (8, False), (1, True)])
def test_pipelined_reverse_sweep_is_bit_identical(n, pen, monkeypatch):
    """Small batches recompute the checkpoint segments on two wavefronts per
    workgroup and run the reverse sweep as a pipeline on four (motor re-run,
    body re-run, contacts, derivative); the gradients equal those of the
    one-wavefront kernels bit for bit."""
    w, acts, Wt, gpen = problem(7, 12, n_envs=20 if n == 8 else 150, n=n, spread=0.6)
    gp = gpen if pen else None
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("QS_REVERSE_PIPE", mode)
        monkeypatch.setenv("QS_RECOMPUTE_PIPE", mode)
        sim = QuadSwarm.from_workload(w)
        a = dev(acts)
        ckpt = torch.empty((3, 27, w.n_quads), device="cuda")
        pen_t = torch.zeros(w.n_quads, device="cuda") if pen else None
        sim.rollout(a, 2, 5, ckpt, pen_t, BETA if pen else 0.0)
        gs = dev(Wt).clone()
        gact = torch.empty_like(a)
        gpar = torch.zeros((w.n_quads, 6), device="cuda")
        sim.rollout_backward(a, 2, 5, ckpt, 0, gs, None if gp is None else dev(gp),
                             BETA if pen else 0.0, gact, gpar)
        sim.sync()
        out[mode] = (gs.cpu(), gact.cpu(), gpar.cpu())
        sim.close()
    for x, y in zip(out["0"], out["1"]):
        assert torch.equal(x, y)
    assert float(out["1"][1].abs().max()) > 0


@pytest.mark.parametrize("n,pen", [(8, True), (8, False), (1, False)])
def test_pipelined_rollout_is_bit_identical(n, pen, monkeypatch):
    """Small batches run the rollout in two wavefronts per workgroup (the
    motor part one substep ahead); state, checkpoints and penalty equal the
    one-wavefront rollout bit for bit."""
    w, acts, Wt, gpen = problem(8, 13, n_envs=20 if n == 8 else 150, n=n, spread=0.6)
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("QS_ROLLOUT_PIPE", mode)
        sim = QuadSwarm.from_workload(w)
        ckpt = torch.empty((3, 27, w.n_quads), device="cuda")
        pen_t = torch.zeros(w.n_quads, device="cuda") if pen else None
        sim.rollout(dev(acts), 3, 5, ckpt, pen_t, BETA if pen else 0.0)
        sT, tT = sim.get_state()
        sim.sync()
        out[mode] = (sT.cpu(), ckpt.cpu(), None if pen_t is None else pen_t.cpu(), tT)
        sim.close()
    assert out["0"][3] == out["1"][3] == 13 * 3
    assert torch.equal(out["0"][0], out["1"][0])
    assert torch.equal(out["0"][1], out["1"][1])
    if pen:
        assert torch.equal(out["0"][2], out["1"][2]) and float(out["1"][2].max()) > 0


def test_step_backward_matches_oracle():
    w, acts, Wt, gpen = problem(5, 1)
    nsub = 3
    sim = QuadSwarm.from_workload(w)
    s_in, _ = sim.get_state()
    gin = torch.empty((w.n_quads, 27), device="cuda")
    gact = torch.empty((w.n_quads, 4), device="cuda")
    gpar = torch.zeros((w.n_quads, 6), device="cuda")
    sim.step_backward(s_in, dev(acts[0]), nsub, 0, dev(Wt), gin, gact, gpar)
    sim.sync()
    orc = O.Oracle.from_workload(w)
    s0 = w.state0.astype(np.float64)
    ref = orc.rollout_vjp(s0, acts.astype(np.float64), nsub, 0, Wt.astype(np.float64), None, None)
    rng = np.random.default_rng(5)
    s0p = s0 * (1 + rng.uniform(-1, 1, size=s0.shape) * 2.0 ** -23)
    pert = orc.rollout_vjp(s0p, acts.astype(np.float64), nsub, 0, Wt.astype(np.float64), None,
                           None)
    check((gin.cpu().numpy(), gact.cpu().numpy()[None], gpar.cpu().numpy()), ref, pert,
          "qs_step_backward")


def test_autograd_function_matches_direct_calls():
    w, acts, Wt, gpen = problem(2, 12)
    sim = QuadSwarm.from_workload(w)
    s0 = dev(w.state0).requires_grad_(True)
    a = dev(acts).requires_grad_(True)
    p = dev(w.params).requires_grad_(True)
    sT, pen = rollout(sim, s0, a, p, n_substeps=2, ckpt_every=4, beta=BETA)
    loss = (sT * dev(Wt)).sum() + (pen * dev(gpen)).sum()
    loss.backward()
    gs, gact, gpar, *_ = gpu_grads(w, acts, 2, Wt, gpen, 4)
    np.testing.assert_allclose(s0.grad.cpu().numpy(), gs, rtol=0, atol=0)
    np.testing.assert_allclose(a.grad.cpu().numpy(), gact, rtol=0, atol=0)
    np.testing.assert_allclose(p.grad.cpu().numpy(), gpar, rtol=0, atol=0)


def test_checkpoint_interval_does_not_change_gradients():
    """Recomputation from checkpoints reproduces the forward bit for bit, so
    state and action gradients are identical for any checkpoint interval;
    parameter gradients are summed per segment, so only their rounding
    (summation grouping) may differ."""
    w, acts, Wt, gpen = problem(4, 40)
    g1 = gpu_grads(w, acts, 1, Wt, gpen, 40)
    g2 = gpu_grads(w, acts, 1, Wt, gpen, 7)
    np.testing.assert_array_equal(g1[0], g2[0])
    np.testing.assert_array_equal(g1[1], g2[1])
    np.testing.assert_allclose(g1[2], g2[2], rtol=1e-5, atol=1e-6 * np.abs(g1[2]).max())


def test_diff_workload_full_size_sampled():
    """1024 envs x 8 quads, 200-substep horizon, checkpoint every 20 calls:
    envs 100..103 checked against the oracle's derivative."""
    w = W.diff(seed=0)
    T, nsub, ce = 200, 1, 20
    rng = np.random.default_rng(9)
    acts = rng.uniform(0.05, 0.95, size=(T, w.n_quads, 4)).astype(np.float32)
    Wt = rng.normal(size=(w.n_quads, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = rng.uniform(0.5, 2.0, size=w.n_quads).astype(np.float32)
    gs, gact, gpar, *_ = gpu_grads(w, acts, nsub, Wt, gpen, ce)
    assert np.isfinite(gs).all() and np.isfinite(gact).all() and np.isfinite(gpar).all()
    e0, e1 = 100, 104
    q0, q1 = int(w.env_offsets[e0]), int(w.env_offsets[e1])
    g_ref = oracle_grads(w, acts, nsub, Wt, gpen, env_range=(e0, e1))
    g_pert = oracle_pert(w, acts, nsub, Wt, gpen, 9, env_range=(e0, e1))
    check((gs[q0:q1], gact[:, q0:q1], gpar[q0:q1]), g_ref, g_pert, "1024 x 8 sampled")


def floor_wall_problem(**c):
    """Eight quads resting (some sliding) on the floor under low thrust and
    eight flying into the +x wall: the floor-rest, friction and wall-mirror
    branches of the adjoint (the oracle's own pin of these branches, on the
    GPU)."""
    w, s0 = dense_problem(11, n_envs=2, z=0.0, spread=0.3, **c)
    s0[:, 2] = 0.0
    s0[:, W.SF] = 1.0
    s0[:, W.SR:W.SR + 9] = np.eye(3).reshape(9)
    s0[:8, W.SV:W.SV + 2] = np.random.default_rng(1).normal(0, 0.5, size=(8, 2))
    s0[8:, 0] = 4.95
    s0[8:, W.SF] = 0.0
    s0[8:, 2] = 3.0
    s0[8:, W.SV] = 2.0
    w = w.with_(state0=s0.astype(np.float32))
    rng = np.random.default_rng(5)
    T = 10
    acts = np.concatenate([rng.uniform(0.0, 0.2, size=(T, 8, 4)) - 0.8,
                           rng.uniform(0.2, 0.8, size=(T, 8, 4))], axis=1).astype(np.float32)
    Wt = rng.normal(size=(w.n_quads, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = np.ones(w.n_quads, np.float32)
    return w, acts, Wt, gpen


@pytest.mark.parametrize("c", [{}, LOSSY])
def test_adjoint_through_floor_and_walls_matches_oracle(c):
    """Gradients through floor rest and friction and the wall mirror; with
    non-default constants also through the drag, decay and restitution
    terms."""
    w, acts, Wt, gpen = floor_wall_problem(**c)
    g_ref = oracle_grads(w, acts, 1, Wt, gpen)
    g_pert = oracle_pert(w, acts, 1, Wt, gpen, 11)
    gs, gact, gpar, sT, *_ = gpu_grads(w, acts, 1, Wt, gpen, 4)
    assert np.all(sT[:8, W.SF] == 1.0) and np.all(sT[8:, 0] <= 5.0)
    check((gs, gact, gpar), g_ref, g_pert, "floor/wall adjoint")


def test_adjoint_through_floor_hits_matches_oracle():
    """64 tilted, yawed quads land in the first substep (the attitude levelled
    keeping the heading) and then rest under low thrust: the floor-hit branch
    of the adjoint on the GPU against the oracle's."""
    from tests.helpers import rot_x, rot_z
    n = 64
    w = W.custom([1] * n, seed=32, k=0, flags=W.QS_FLOOR | W.QS_MOTOR_NOISE, name="land")
    rng = np.random.default_rng(32)
    s0 = w.state0.astype(np.float64).copy()
    s0[:, 0:2] = rng.uniform(-3, 3, size=(n, 2))
    s0[:, 2] = rng.uniform(0.001, 0.004, n)
    s0[:, W.SV:W.SV + 3] = np.column_stack([rng.uniform(-0.3, 0.3, (n, 2)), np.full(n, -1.0)])
    for q in range(n):
        s0[q, W.SR:W.SR + 9] = (rot_z(rng.uniform(-3, 3)) @ rot_x(rng.uniform(0.1, 0.5))).reshape(9)
    s0[:, W.SW:W.SW + 3] = rng.normal(0, 0.4, size=(n, 3))
    s0[:, W.SF] = 0.0
    w = w.with_(state0=s0.astype(np.float32))
    T = 4
    acts = np.full((T, n, 4), -0.9, np.float32)
    Wt = rng.normal(size=(n, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = np.zeros(n, np.float32)
    g_ref = oracle_grads(w, acts, 1, Wt, gpen)
    g_pert = oracle_pert(w, acts, 1, Wt, gpen, 32)
    gs, gact, gpar, sT, *_ = gpu_grads(w, acts, 1, Wt, gpen, 2)
    assert np.all(sT[:, W.SF] == 1.0)
    check((gs, gact, gpar), g_ref, g_pert, "floor-hit adjoint")


def test_adjoint_through_static_friction_breakaway_matches_oracle():
    """64 resting quads tilted 20-35 degrees about body y (random heading),
    horizontal thrust above mu N: the first substep takes the static branch
    of the floor friction, the later ones the kinetic branch.  GPU gradients
    against the oracle's."""
    import math
    from tests.helpers import rot_y, rot_z
    n = 64
    w = W.custom([1] * n, seed=34, k=0, flags=W.QS_FLOOR, randomise=False, name="slide")
    rng = np.random.default_rng(34)
    s0 = w.state0.astype(np.float64).copy()
    s0[:, 0:2] = rng.uniform(-3, 3, size=(n, 2))
    s0[:, 2] = 0.0
    s0[:, W.SV:W.SV + 3] = 0.0
    s0[:, W.SF] = 1.0
    for q in range(n):
        R = rot_z(rng.uniform(-3, 3)) @ rot_y(math.radians(rng.uniform(20, 35)))
        s0[q, W.SR:W.SR + 9] = R.reshape(9)
    s0[:, W.SW:W.SW + 3] = 0.0
    s0[:, W.SU:W.SU + 4] = math.sqrt(0.45)
    s0[:, W.SE:W.SE + 4] = 0.0
    w = w.with_(state0=s0.astype(np.float32))
    T = 4
    acts = np.full((T, n, 4), -0.1, np.float32)
    Wt = rng.normal(size=(n, 27)).astype(np.float32)
    Wt[:, 26] = 0
    gpen = np.zeros(n, np.float32)
    g_ref = oracle_grads(w, acts, 1, Wt, gpen)
    g_pert = oracle_pert(w, acts, 1, Wt, gpen, 34)
    gs, gact, gpar, sT, *_ = gpu_grads(w, acts, 1, Wt, gpen, 2)
    assert np.all(sT[:, W.SF] == 1.0) and np.all(np.hypot(sT[:, W.SV], sT[:, W.SV + 1]) > 0)
    check((gs, gact, gpar), g_ref, g_pert, "static-friction adjoint")
