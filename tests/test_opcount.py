"""The op-counting build of the oracle (oracle/opcount.cpp), CPU.

It must compute exactly what the oracle computes (bitwise equal results),
and its counts must be the operation counts of the definition, checked
against counts derived by hand from the equations:

- one free-flight substep of a single quad without noise, room or floor:
  action map 8 + 4 square roots, lag 12, thrust 12, mix 3 + 12, world
  thrust 3, acceleration 13, Euler's equation 18, semi-implicit Euler 18,
  attitude update 72, Gram-Schmidt 36 + 2 square roots, cross product 9:
  207 add/mul/div (15 of them divisions) and 6 square roots;
- motor noise adds two Box-Muller pairs (14 multiplies, 2 square roots,
  6 transcendentals) and the AR(1) update (12): 34 operations;
- a pair test without contact is a squared distance, 8 operations;
- an observation is 3 (goal offset) + 8 per swarm-mate distance (self
  included) + 6 per filled neighbour slot.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_09537_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import json, sys
import numpy as np
sys.path.insert(0, ROOT)
from oracle import oracle as O
from paper_2306_09537_amd import workloads as W
from tests.test_opcount import cases
out = {}
for name, (w, nsub) in cases().items():
    orc = O.Oracle.from_workload(w)
    s0 = w.state0.astype(np.float64)
    O.opcount_reset()
    s, _, _ = orc.step(s0, w.actions(0).astype(np.float64), nsub, 0)
    st = O.opcount_get()
    O.opcount_reset()
    obs, _ = orc.observe(s, w.goals.astype(np.float64))
    ob = O.opcount_get()
    g = orc.rollout_vjp(s0, w.action_sequence(3).astype(np.float64), 1, 0,
                        np.ones((w.n_quads, 27)), np.ones(w.n_quads), 100.0)
    out[name] = dict(step=st, observe=ob, s=s.tolist(), obs=obs.tolist(),
                     g=[a.tolist() for a in g])
print(json.dumps(out))
'''


def spread(w, gap=3.0):
    """Quads of every swarm on a line gap/10 m apart, far from walls and
    floor: no contacts, no events."""
    s = w.state0.copy()
    for e in range(w.n_envs):
        q0, q1 = int(w.env_offsets[e]), int(w.env_offsets[e + 1])
        for i, q in enumerate(range(q0, q1)):
            s[q, 0:3] = [-4.0 + 0.02 * e, -4.0 + gap / 10 * i, 5.0]
    return w.with_(state0=s)


def cases():
    return {
        "free": (W.custom([1] * 8, seed=1, k=0, flags=0, name="free"), 1),
        "noise": (W.custom([1] * 8, seed=2, k=0, flags=W.QS_MOTOR_NOISE, name="noise"), 1),
        "pairs5": (spread(W.custom([5] * 4, seed=3, k=3, flags=W.QS_COLLIDE, name="p5")), 1),
        "single5": (spread(W.custom([1] * 20, seed=3, k=3, flags=W.QS_COLLIDE, name="s5")), 1),
        "swarm8": (W.custom([8] * 16, seed=4, k=6, name="swarm8"), 3),
    }


@pytest.fixture(scope="module")
def counted():
    O.build_opcount()
    env = dict(os.environ, QS_ORACLE_LIB=O.OPCOUNT_LIB)
    code = "ROOT = %r\n" % ROOT + SCRIPT
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300, check=True)
    return json.loads(p.stdout)


def test_counting_build_computes_what_the_oracle_computes(counted):
    for name, (w, nsub) in cases().items():
        orc = O.Oracle.from_workload(w)
        s0 = w.state0.astype(np.float64)
        s, _, _ = orc.step(s0, w.actions(0).astype(np.float64), nsub, 0)
        obs, _ = orc.observe(s, w.goals.astype(np.float64))
        g = orc.rollout_vjp(s0, w.action_sequence(3).astype(np.float64), 1, 0,
                            np.ones((w.n_quads, 27)), np.ones(w.n_quads), 100.0)
        c = counted[name]
        np.testing.assert_array_equal(np.array(c["s"]), s)
        np.testing.assert_array_equal(np.array(c["obs"]), obs)
        for a, b in zip(c["g"], g):
            np.testing.assert_array_equal(np.array(a), b)


def test_free_flight_substep_count(counted):
    st = counted["free"]["step"]
    q = 8
    assert st["add"] + st["mul"] + st["div"] == 207 * q
    assert st["div"] == 15 * q and st["sqrt"] == 6 * q and st["trans"] == 0


def test_motor_noise_count(counted):
    a, b = counted["free"]["step"], counted["noise"]["step"]
    q = 8
    assert b["total"] - a["total"] == 34 * q
    assert b["trans"] - a["trans"] == 6 * q and b["sqrt"] - a["sqrt"] == 2 * q


def test_pair_test_count(counted):
    # 4 swarms of 5: 10 pair tests each, no contact; against the same 20
    # quads stepped as single-quad swarms
    diff = counted["pairs5"]["step"]["total"] - counted["single5"]["step"]["total"]
    assert diff == 4 * 10 * 8


@pytest.mark.parametrize("name,n,k,q", [("free", 1, 0, 8), ("pairs5", 5, 3, 20),
                                        ("swarm8", 8, 6, 128)])
def test_observation_count(counted, name, n, k, q):
    assert counted[name]["observe"]["total"] == q * (3 + 8 * n + 6 * min(k, n - 1))
