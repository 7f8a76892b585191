"""Pins of the oracle's reverse-mode derivative against FP64 central
differences (h = 1e-6) of the oracle's own forward rollout.

Loss: L = sum_q,k W[q,k] s_T[q,k] + sum_q gpen[q] pen[q], with random weights
W (the resting flag excluded) and gpen, where pen is each quad's share of
the softplus-smoothed collision penalty.  Small dense swarms make contacts,
collision responses and penalty gradients all active; seeds are chosen so
that no event sits within the perturbation of its threshold.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_09537_amd import workloads as W

BETA = 100.0


def dense_problem(seed, n_envs=4, n=8, spread=0.25, flags=W.SWARM_FLAGS, z=3.0, **c):
    w = W.custom([n] * n_envs, seed=seed, k=6, flags=flags, name="grad", **c)
    rng = np.random.default_rng(seed)
    s0 = w.state0.astype(np.float64).copy()
    for e in range(n_envs):
        s0[e * n:(e + 1) * n, 0:3] = rng.uniform(-2, 2, 3) * [1, 1, 0] + [0, 0, z] + \
            rng.uniform(-spread, spread, size=(n, 3))
    return w, s0


def loss(orc, s0, acts, nsub, Wt, gpen):
    sT, pen = orc.rollout(s0, acts, nsub, 0, beta=BETA)
    return float(np.sum(Wt * sT) + np.sum(gpen * pen))


def setup(seed, T, nsub, **kw):
    w, s0 = dense_problem(seed, **kw)
    orc = O.Oracle.from_workload(w)
    rng = np.random.default_rng(seed + 100)
    acts = rng.uniform(0.05, 0.95, size=(T, w.n_quads, 4))
    Wt = rng.normal(size=(w.n_quads, 27))
    Wt[:, 26] = 0.0
    gpen = rng.uniform(0.5, 2.0, size=w.n_quads)
    gs0, gact, gpar = orc.rollout_vjp(s0, acts, nsub, 0, Wt, gpen, BETA)
    return w, s0, orc, acts, Wt, gpen, gs0, gact, gpar


def fd(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


# non-default constants make the drag, wall-restitution and decay terms of
# the reverse mode count (at the defaults they vanish or are the identity)
LOSSY = dict(drag_coef=0.05, col_decay=0.9, wall_restitution=0.8)


@pytest.mark.parametrize("seed,c", [(0, {}), (1, {}), (2, LOSSY)])
def test_action_gradient_matches_central_differences(seed, c):
    T, nsub = 30, 2
    w, s0, orc, acts, Wt, gpen, gs0, gact, gpar = setup(seed, T, nsub, **c)
    rng = np.random.default_rng(seed)
    h = 1e-6
    checked = 0
    for _ in range(24):
        c, q, i = rng.integers(T), rng.integers(w.n_quads), rng.integers(4)

        def f(v):
            a = acts.copy()
            a[c, q, i] = v
            return loss(orc, s0, a, nsub, Wt, gpen)
        g = fd(f, acts[c, q, i], h)
        assert gact[c, q, i] == pytest.approx(g, rel=2e-5, abs=1e-7 * (1 + abs(g))), (c, q, i)
        checked += 1
    assert checked == 24


@pytest.mark.parametrize("seed", [0, 3])
def test_param_gradient_matches_central_differences(seed):
    T, nsub = 30, 2
    w, s0, orc, acts, Wt, gpen, gs0, gact, gpar = setup(seed, T, nsub)
    P = orc.params
    for q in (0, 5, 13, 30):
        for k in range(6):
            h = 1e-6 * P[q, k]

            def f(v):
                p2 = P.copy()
                p2[q, k] = v
                return loss(orc.with_params(p2), s0, acts, nsub, Wt, gpen)
            g = fd(f, P[q, k], h)
            assert gpar[q, k] == pytest.approx(g, rel=2e-5, abs=1e-6 * (1 + abs(g))), (q, k)


def test_initial_state_gradient_matches_central_differences():
    T, nsub = 20, 1
    w, s0, orc, acts, Wt, gpen, gs0, gact, gpar = setup(7, T, nsub)
    rng = np.random.default_rng(7)
    for _ in range(30):
        q, k = rng.integers(w.n_quads), rng.integers(26)
        h = 1e-7

        def f(v):
            s = s0.copy()
            s[q, k] = v
            return loss(orc, s, acts, nsub, Wt, gpen)
        g = fd(f, s0[q, k], h)
        assert gs0[q, k] == pytest.approx(g, rel=5e-5, abs=1e-6 * (1 + abs(g))), (q, k)


def test_contacts_and_penalty_are_exercised():
    """The dense setup really has collision responses and penalty gradient."""
    w, s0 = dense_problem(0)
    orc = O.Oracle.from_workload(w)
    acts = np.random.default_rng(100).uniform(0.05, 0.95, size=(30, w.n_quads, 4))
    s, responded = s0, 0
    for c in range(30):
        s, contacts, ev = orc.step(s, acts[c], 2, 2 * c)
        responded += int(np.count_nonzero(ev & O.EV_PAIR_RESPONSE))
    assert responded > 5
    _, pen = orc.rollout(s0, acts, 2, 0, beta=BETA)
    assert pen.min() > 0 and pen.max() > 1e-3


@pytest.mark.parametrize("c", [{}, LOSSY])
def test_floor_and_wall_branches(c):
    """Gradients through the floor rest / friction and the wall mirror."""
    w, s0 = dense_problem(11, n_envs=2, z=0.0, spread=0.3, **c)
    s0[:, 2] = 0.0
    s0[:, W.SF] = 1.0                       # resting
    s0[:, W.SR:W.SR + 9] = np.eye(3).reshape(9)
    s0[:8, W.SV:W.SV + 2] = np.random.default_rng(1).normal(0, 0.5, size=(8, 2))  # sliding
    s0[8:, 0] = 4.95                         # near the +x wall
    s0[8:, W.SF] = 0.0
    s0[8:, 2] = 3.0
    s0[8:, W.SV] = 2.0
    orc = O.Oracle.from_workload(w)
    rng = np.random.default_rng(5)
    T, nsub = 10, 1
    acts = np.concatenate([rng.uniform(0.0, 0.2, size=(T, 8, 4)) - 0.8,
                           rng.uniform(0.2, 0.8, size=(T, 8, 4))], axis=1)
    Wt = rng.normal(size=(w.n_quads, 27))
    Wt[:, 26] = 0
    gpen = np.ones(w.n_quads)
    sT, _ = orc.rollout(s0, acts, nsub, 0, beta=BETA)
    assert np.all(sT[:8, W.SF] == 1.0)       # stayed on the floor
    gs0, gact, gpar = orc.rollout_vjp(s0, acts, nsub, 0, Wt, gpen, BETA)
    for q, k in [(0, 3), (1, 4), (2, 0), (9, 3), (10, 0), (12, 1)]:
        h = 1e-7

        def f(v):
            s = s0.copy()
            s[q, k] = v
            return loss(orc, s, acts, nsub, Wt, gpen)
        assert gs0[q, k] == pytest.approx(fd(f, s0[q, k], h), rel=5e-5, abs=1e-6)
    for q in (0, 3, 9):
        for k in (0, 4):
            P = orc.params
            h = 1e-6 * P[q, k]

            def f(v):
                p2 = P.copy()
                p2[q, k] = v
                return loss(orc.with_params(p2), s0, acts, nsub, Wt, gpen)
            assert gpar[q, k] == pytest.approx(fd(f, P[q, k], h), rel=5e-5, abs=1e-6)


def test_floor_hit_gradient_through_the_levelled_heading():
    """Tilted, yawed quads land in the first substep: the attitude is levelled
    keeping the heading (R = [h, e_z x h, e_z], h the normalised (R00, R10)
    after the substep's rotation update), so the final attitude depends on
    the initial one only through that heading.  The adjoint of the levelling
    (the normalisation's projection included) against central differences."""
    from tests.helpers import rot_x, rot_z
    w = W.custom([1, 1], seed=31, k=0, flags=W.QS_FLOOR, name="land")
    s0 = w.state0.astype(np.float64).copy()
    for q, (psi, tilt) in enumerate([(0.7, 0.4), (-2.0, 0.25)]):
        s0[q, 0:3] = [0.0, 0.0, 0.004]
        s0[q, W.SV:W.SV + 3] = [0.2, -0.1, -1.0]
        s0[q, W.SR:W.SR + 9] = (rot_z(psi) @ rot_x(tilt)).reshape(9)
        s0[q, W.SW:W.SW + 3] = [0.3, -0.2, 0.5]
        s0[q, W.SF] = 0.0
    orc = O.Oracle.from_workload(w)
    acts = np.full((2, 2, 4), -1.0)
    rng = np.random.default_rng(31)
    Wt = rng.normal(size=(2, 27))
    Wt[:, 26] = 0.0
    gpen = np.zeros(2)
    sT, _ = orc.rollout(s0, acts, 1, 0, beta=BETA)
    assert np.all(sT[:, W.SF] == 1.0)
    gs0, _, _ = orc.rollout_vjp(s0, acts, 1, 0, Wt, gpen, BETA)
    biggest = 0.0
    for q in range(2):
        for k in (W.SR + 0, W.SR + 1, W.SR + 3, W.SR + 4, W.SW + 0, W.SW + 2):
            def f(v):
                s = s0.copy()
                s[q, k] = v
                return loss(orc, s, acts, 1, Wt, gpen)
            g = fd(f, s0[q, k], 1e-7)
            biggest = max(biggest, abs(g))
            assert gs0[q, k] == pytest.approx(g, rel=1e-5, abs=1e-7), (q, k)
    assert biggest > 0.1          # the heading carries real sensitivity


def test_static_friction_breakaway_gradient():
    """Resting quads tilted about body y, horizontal thrust above mu N, start
    to slide from rest: their first substep takes the static branch (force
    |F_xy| - mu N along F_xy), the later ones the kinetic branch.  Gradients
    with respect to the attitude's third column, the rotor speed, an action
    and the parameters against central differences."""
    import math
    from tests.helpers import rot_y, rot_z
    w = W.custom([1, 1], seed=33, k=0, flags=W.QS_FLOOR, randomise=False, name="slide")
    s0 = w.state0.astype(np.float64).copy()
    for q, (theta, psi) in enumerate([(30.0, 0.3), (25.0, -1.1)]):
        s0[q, 0:3] = [0.5 * q, 0.0, 0.0]
        s0[q, W.SV:W.SV + 3] = 0.0
        s0[q, W.SF] = 1.0
        s0[q, W.SR:W.SR + 9] = (rot_z(psi) @ rot_y(math.radians(theta))).reshape(9)
        s0[q, W.SW:W.SW + 3] = 0.0
        s0[q, W.SU:W.SU + 4] = math.sqrt(0.45)
        s0[q, W.SE:W.SE + 4] = 0.0
    orc = O.Oracle.from_workload(w)
    acts = np.full((3, 2, 4), -0.1)                 # normalised thrust 0.45
    rng = np.random.default_rng(33)
    Wt = rng.normal(size=(2, 27))
    Wt[:, 26] = 0.0
    gpen = np.zeros(2)
    sT, _ = orc.rollout(s0, acts, 1, 0, beta=BETA)
    assert np.all(sT[:, W.SF] == 1.0) and np.all(np.abs(sT[:, W.SV]) + np.abs(sT[:, W.SV + 1]) > 0)
    gs0, gact, gpar = orc.rollout_vjp(s0, acts, 1, 0, Wt, gpen, BETA)
    for q in range(2):
        for k in (W.SR + 2, W.SR + 5, W.SR + 8, W.SU + 0):
            def f(v):
                s = s0.copy()
                s[q, k] = v
                return loss(orc, s, acts, 1, Wt, gpen)
            assert gs0[q, k] == pytest.approx(fd(f, s0[q, k], 1e-7), rel=1e-5, abs=1e-8), (q, k)

        def fa(v):
            a = acts.copy()
            a[0, q, 1] = v
            return loss(orc, s0, a, 1, Wt, gpen)
        assert gact[0, q, 1] == pytest.approx(fd(fa, acts[0, q, 1], 1e-7), rel=1e-5, abs=1e-8)
        for k in (0, 4):
            P = orc.params
            h = 1e-6 * P[q, k]

            def fp(v):
                p2 = P.copy()
                p2[q, k] = v
                return loss(orc.with_params(p2), s0, acts, 1, Wt, gpen)
            assert gpar[q, k] == pytest.approx(fd(fp, P[q, k], h), rel=1e-5, abs=1e-8), (q, k)


@pytest.mark.slow
def test_200_step_horizon_action_gradient():
    """The differentiation workload's horizon: 200 substeps, 4 envs x 8 quads."""
    T, nsub = 200, 1
    w, s0, orc, acts, Wt, gpen, gs0, gact, gpar = setup(2, T, nsub, spread=0.4)
    rng = np.random.default_rng(2)
    for _ in range(10):
        c, q, i = rng.integers(150, T), rng.integers(w.n_quads), rng.integers(4)

        def f(v):
            a = acts.copy()
            a[c, q, i] = v
            return loss(orc, s0, a, nsub, Wt, gpen)
        g = fd(f, acts[c, q, i], 1e-6)
        assert gact[c, q, i] == pytest.approx(g, rel=1e-4, abs=1e-6 * (1 + abs(g)))


def test_rollout_matches_repeated_steps():
    w, s0 = dense_problem(4)
    orc = O.Oracle.from_workload(w)
    acts = np.random.default_rng(4).uniform(0, 1, size=(6, w.n_quads, 4))
    sT, _ = orc.rollout(s0, acts, 3, 10)
    s = s0
    for c in range(6):
        s, _, _ = orc.step(s, acts[c], 3, 10 + 3 * c)
    assert np.array_equal(s, sT)
