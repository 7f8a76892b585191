"""The seeded input generator: shapes, determinism and the stated distributions."""
import math

import numpy as np

from paper_2306_09537_amd import workloads as W


def test_shapes_and_determinism():
    for name, fn in W.WORKLOADS.items():
        small = {"plain": 8, "swarm8": 16, "uneven": 32, "diff": 8, "scale32": 2, "scale1": 64}[name]
        a, b = fn(seed=1, n_envs=small), fn(seed=1, n_envs=small)
        q = a.n_quads
        assert a.params.shape == (q, 6) and a.state0.shape == (q, 27) and a.goals.shape == (q, 3)
        assert a.params.dtype == np.float32 and a.state0.dtype == np.float32
        assert np.array_equal(a.state0, b.state0) and np.array_equal(a.params, b.params)
        assert np.array_equal(a.actions(3), b.actions(3))
        assert not np.array_equal(a.actions(3), a.actions(4))
        assert a.env_offsets[0] == 0 and np.all(np.diff(a.env_offsets) == a.env_sizes)
        assert np.all((a.env_sizes >= 1) & (a.env_sizes <= 32))


def test_initial_state_distribution():
    w = W.swarm8(seed=2, n_envs=512)
    s = w.state0.astype(np.float64)
    R = s[:, W.SR:W.SR + 9].reshape(-1, 3, 3)
    assert np.abs(np.einsum("qki,qkj->qij", R, R) - np.eye(3)).max() < 1e-6
    tilt = np.degrees(np.arccos(np.clip(R[:, 2, 2], -1, 1)))
    assert tilt.max() <= 30.0 + 1e-3 and tilt.max() > 25.0
    assert np.all(np.abs(s[:, 0:2]) <= 2.0) and np.all((s[:, 2] >= 0.5) & (s[:, 2] <= 2.5))
    assert abs(s[:, W.SV:W.SV + 3].std() - 0.5) < 0.03
    np.testing.assert_allclose(s[:, W.SU], np.sqrt(1.0 / w.params[:, 4]), rtol=1e-6)
    assert np.all(s[:, W.SE:] == 0.0)


def test_domain_randomisation_ranges():
    w = W.swarm8(seed=0, n_envs=1024)
    nom = np.array([W.NOMINAL[k] for k in ("mass", "ixx", "iyy", "izz", "thrust_to_weight", "motor_tau")])
    r = w.params / nom
    assert np.all((r[:, :5] >= 0.8 - 1e-6) & (r[:, :5] <= 1.2 + 1e-6))
    assert np.all((r[:, 5] >= 0.7 - 1e-6) & (r[:, 5] <= 1.3 + 1e-6))
    assert r[:, 0].std() > 0.1
    p = W.plain(n_envs=4).params
    assert np.allclose(p / nom, 1.0)


def test_uneven_sizes_cover_buckets():
    w = W.uneven(seed=0, n_envs=2048)
    assert set(np.unique(w.env_sizes)) == {1, 2, 4, 8, 16, 32}
    assert abs(w.n_quads / 2048 - 63 / 6) < 1.0


def test_actions_range():
    w = W.swarm8(n_envs=64)
    a = w.actions(0)
    assert a.min() >= 0.0 and a.max() <= 1.0 and abs(a.mean() - 0.5) < 0.02
    seq = w.action_sequence(3)
    assert seq.shape == (3, w.n_quads, 4) and seq.min() >= 0 and seq.max() <= 1
