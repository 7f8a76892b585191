"""The block-wise gradient check (tests/grad_check.py) on oracle data, CPU.

The GPU gradient tests compare each block of the float32 gradient (state
field groups, rotors, each parameter column) with the oracle's on its own
scale.  Here the check itself is pinned: a second, independent float32-sized
perturbation of the oracle's input passes it, while the gradient with any
one block zeroed, a parameter column off by 1 %, or a column with its sign
flipped fails it, even for the columns that carry a tiny share of the
parameter gradient's norm (thrust-to-weight, tau_m, mass)."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import grad_check as G
from tests.test_oracle_grad import BETA, dense_problem


@pytest.fixture(scope="module")
def grads():
    w, s0 = dense_problem(0)
    orc = O.Oracle.from_workload(w)
    rng = np.random.default_rng(100)
    T, nsub = 30, 2
    acts = rng.uniform(0.05, 0.95, size=(T, w.n_quads, 4))
    Wt = rng.normal(size=(w.n_quads, 27))
    Wt[:, 26] = 0.0
    gpen = rng.uniform(0.5, 2.0, size=w.n_quads)

    def g(s):
        return orc.rollout_vjp(s, acts, nsub, 0, Wt, gpen, BETA)

    s32 = s0.astype(np.float32).astype(np.float64)
    ref = g(s32)
    p1 = g(s32 * (1 + np.random.default_rng(1).uniform(-1, 1, s32.shape) * 2.0 ** -23))
    p2 = g(s32 * (1 + np.random.default_rng(2).uniform(-1, 1, s32.shape) * 2.0 ** -23))
    return ref, p1, p2


def test_small_columns_are_tiny_shares_of_the_norm(grads):
    """Why the check is block-wise: a norm over all six parameter columns
    would not see the thrust-to-weight, tau_m or mass columns."""
    gp = grads[0][2]
    share = np.linalg.norm(gp, axis=0) / np.linalg.norm(gp)
    assert share[4] < 1e-3 and share[5] < 1e-3 and share[0] < 1e-2


def test_independent_rounding_perturbation_passes(grads):
    ref, p1, p2 = grads
    rows = G.compare(p2, ref, p1)
    assert not G.failures(rows), G.report(rows, "perturbation")


@pytest.mark.parametrize("block", [b for b, _ in G.blocks(*[np.zeros((2, 27)), np.zeros((1, 2, 4)),
                                                             np.zeros((2, 6))])])
def test_zeroed_block_fails(grads, block):
    ref, p1, p2 = grads
    bad = G.zeroed(p2, block)
    failed = [r[0] for r in G.failures(G.compare(bad, ref, p1))]
    assert failed == [block]


@pytest.mark.parametrize("col", range(6))
def test_parameter_column_off_by_one_percent_or_flipped_fails(grads, col):
    ref, p1, p2 = grads
    for factor in (1.01, -1.0):
        gp = np.array(p2[2], copy=True)
        gp[:, col] *= factor
        failed = [r[0] for r in G.failures(G.compare((p2[0], p2[1], gp), ref, p1))]
        assert failed == ["param." + G.PARAM_NAMES[col]], (factor, failed)


def test_analytically_zero_block_allows_float32_noise_only(grads):
    """A reference block that is zero to double precision (the mass column
    of quads resting on the floor) passes with float32-sized noise in the
    float32 gradient and fails with anything larger."""
    ref, p1, p2 = grads
    rng = np.random.default_rng(3)
    fam = np.linalg.norm(ref[2])
    gp_ref, gp_pert = np.array(ref[2], copy=True), np.array(p1[2], copy=True)
    gp_ref[:, 0] = rng.normal(0, 1e-17, gp_ref.shape[0])
    gp_pert[:, 0] = rng.normal(0, 1e-17, gp_ref.shape[0])
    r0, r1 = (ref[0], ref[1], gp_ref), (p1[0], p1[1], gp_pert)
    for scale, ok in ((1e-7, True), (1e-4, False)):
        gp = np.array(p2[2], copy=True)
        gp[:, 0] = rng.normal(0, 1.0, gp.shape[0])
        gp[:, 0] *= scale * fam / np.linalg.norm(gp[:, 0])
        failed = [r[0] for r in G.failures(G.compare((p2[0], p2[1], gp), r0, r1))]
        assert failed == ([] if ok else ["param.mass"]), (scale, failed)
