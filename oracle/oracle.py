"""ctypes binding of the FP64 oracle (``quadswarm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only users.  Nothing here is imported by the GPU
library, and this file imports nothing from it.

All arrays cross as float64 (state, params, actions, goals), uint64
(contact masks) and uint32 (event bits); the caller's arrays are not
modified except ``state``, which ``step`` returns updated as a new array.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "quadswarm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EV_WALL, EV_FLOOR_HIT, EV_FRICTION, EV_TAKEOFF, EV_PAIR_RESPONSE, EV_CONTACT = 1, 2, 4, 8, 16, 32
EV_DOWNWASH, EV_CEILING = 64, 128


def compile_lib(src: str, out: str) -> None:
    """gcc build of an oracle source file (IEEE double, no FMA contraction)."""
    subprocess.check_call([
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        "-Wno-unused-parameter", src, "-o", out, "-lm"])


def build(force: bool = False) -> str:
    """Compile the oracle into ``liboracle.so`` next to its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        compile_lib(SRC, tmp)
        os.replace(tmp, LIB)
    return LIB


OPCOUNT_SRC = os.path.join(HERE, "opcount.cpp")
OPCOUNT_LIB = os.path.join(HERE, "liboracle_opcount.so")


def build_opcount(force: bool = False) -> str:
    """Compile the op-counting build of the oracle (``opcount.cpp``, which
    includes the oracle's source) into ``liboracle_opcount.so``: single
    threaded, same IEEE double arithmetic, plus or_opcount_reset/get."""
    newest = max(os.path.getmtime(SRC), os.path.getmtime(OPCOUNT_SRC))
    if force or not os.path.exists(OPCOUNT_LIB) or os.path.getmtime(OPCOUNT_LIB) < newest:
        tmp = OPCOUNT_LIB + ".tmp"
        subprocess.check_call([
            "g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wno-unused-parameter", "-Wno-class-memaccess",
            "-Wno-narrowing", "-Wno-unknown-pragmas", OPCOUNT_SRC, "-o", tmp])
        os.replace(tmp, OPCOUNT_LIB)
    return OPCOUNT_LIB


def opcount_reset() -> None:
    """Zero the counters (op-counting build loaded through QS_ORACLE_LIB)."""
    lib().or_opcount_reset()


def opcount_get() -> dict:
    """Counters of the op-counting build since the last reset."""
    o = (C.c_uint64 * 5)()
    lib().or_opcount_get(o)
    add, mul, div, sqrt, trans = (int(v) for v in o)
    return dict(add=add, mul=mul, div=div, sqrt=sqrt, trans=trans,
                total=add + mul + div + sqrt + trans)


class _Desc(C.Structure):
    _fields_ = [
        ("n_envs", C.c_int32), ("env_offsets", C.POINTER(C.c_int32)),
        ("dt", C.c_double), ("gravity", C.c_double), ("arm_length", C.c_double),
        ("k_tau", C.c_double), ("drag_coef", C.c_double), ("floor_mu", C.c_double),
        ("motor_noise_decay", C.c_double), ("motor_noise_std", C.c_double),
        ("room_min", C.c_double * 3), ("room_max", C.c_double * 3),
        ("wall_restitution", C.c_double),
        ("col_dist", C.c_double), ("col_decay", C.c_double),
        ("col_noise_v", C.c_double), ("col_noise_w", C.c_double),
        ("k_neighbors", C.c_int32), ("flags", C.c_uint32), ("seed", C.c_uint64),
        ("quad_id_offset", C.c_uint32),
        ("dw_k1", C.c_double), ("dw_k2", C.c_double), ("dw_b1", C.c_double),
        ("dw_radius", C.c_double), ("dw_height", C.c_double),
        ("dw_noise_a", C.c_double), ("dw_noise_w", C.c_double),
        ("sn_x", C.c_double), ("sn_v", C.c_double), ("sn_w", C.c_double),
    ]


_lib = None


def lib():
    """The loaded oracle.  ``QS_ORACLE_LIB``, when set, names another build
    to load instead: the mutation tests run the pins against copies of the
    source with one planted mistake this way."""
    global _lib
    if _lib is None:
        _lib = C.CDLL(os.environ.get("QS_ORACLE_LIB") or build())
        _lib.or_step.restype = C.c_int
        _lib.or_observe.restype = C.c_int
        _lib.or_uniform_from_u32.restype = C.c_double
        _lib.or_uniform_from_u32.argtypes = [C.c_uint32]
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Oracle:
    """FP64 stepper over one set of environments.

    ``consts`` holds the global constants (dt, gravity, arm_length, k_tau,
    drag_coef, floor_mu, motor_noise_decay, motor_noise_std, room_min,
    room_max, wall_restitution, col_dist, col_decay, col_noise_v,
    col_noise_w); ``params`` is [Q][6] (mass, ixx, iyy, izz,
    thrust_to_weight, motor_tau).
    """

    def __init__(self, env_offsets, consts: dict, params, k_neighbors: int,
                 flags: int, seed: int, quad_id_offset: int = 0):
        self.offs = np.ascontiguousarray(env_offsets, dtype=np.int32)
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.Q = int(self.offs[-1])
        self.K = int(k_neighbors)
        d = _Desc()
        d.n_envs = self.offs.shape[0] - 1
        d.env_offsets = _p(self.offs, C.c_int32)
        for k in ("dt", "gravity", "arm_length", "k_tau", "drag_coef", "floor_mu",
                  "motor_noise_decay", "motor_noise_std", "wall_restitution",
                  "col_dist", "col_decay", "col_noise_v", "col_noise_w"):
            setattr(d, k, float(consts[k]))
        d.room_min = (C.c_double * 3)(*[float(v) for v in consts["room_min"]])
        d.room_max = (C.c_double * 3)(*[float(v) for v in consts["room_max"]])
        d.k_neighbors = self.K
        d.flags = int(flags)
        d.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        d.quad_id_offset = int(quad_id_offset)
        for k in ("dw_k1", "dw_k2", "dw_b1", "dw_radius", "dw_height", "dw_noise_a", "dw_noise_w",
                  "sn_x", "sn_v", "sn_w"):
            setattr(d, k, float(consts.get(k, 0.0)))
        self.desc = d

    @classmethod
    def from_workload(cls, w, env_begin: int = 0, env_end=None) -> "Oracle":
        """Oracle over the environments [env_begin, env_end) of a workload;
        their quads keep their global indices for the noise counters."""
        e1 = w.n_envs if env_end is None else env_end
        offs = w.env_offsets[env_begin:e1 + 1]
        q0, q1 = int(offs[0]), int(offs[-1])
        return cls(offs - q0, w.consts, w.params[q0:q1].astype(np.float64),
                   w.k_neighbors, w.flags, w.rng_key, quad_id_offset=q0)

    def step(self, state, actions, n_sub: int = 1, t0: int = 0, margins: bool = False):
        """Returns (new_state [Q][27] f64, contacts [Q] u64, events [Q] u32),
        plus the per-quad threshold margins [Q] f64 when ``margins``."""
        s = np.array(state, dtype=np.float64, order="C", copy=True)
        a = np.ascontiguousarray(actions, dtype=np.float64)
        assert s.shape == (self.Q, 27) and a.shape == (self.Q, 4)
        contacts = np.zeros(self.Q, dtype=np.uint64)
        events = np.zeros(self.Q, dtype=np.uint32)
        mg = np.zeros(self.Q, dtype=np.float64)
        rc = lib().or_step(C.byref(self.desc), _p(self.params, C.c_double),
                           _p(s, C.c_double), _p(a, C.c_double), C.c_int(n_sub),
                           C.c_uint64(t0), _p(contacts, C.c_uint64),
                           _p(events, C.c_uint32), _p(mg, C.c_double))
        if rc != 0:
            raise ValueError("or_step rejected its arguments")
        if margins:
            return s, contacts, events, mg
        return s, contacts, events

    def rollout(self, state, actions, n_sub: int = 1, t0: int = 0, beta=None):
        """n_calls = actions.shape[0] calls of n_sub substeps.  Returns
        (final state [Q][27], penalty [Q] or None); the penalty is each quad's
        share of sum softplus(beta (d_col - d_ij))/beta over substeps and pairs."""
        s = np.array(state, dtype=np.float64, order="C", copy=True)
        a = np.ascontiguousarray(actions, dtype=np.float64)
        assert a.ndim == 3 and a.shape[1:] == (self.Q, 4)
        pen = np.zeros(self.Q) if beta is not None else None
        rc = lib().or_rollout(C.byref(self.desc), _p(self.params, C.c_double), _p(s, C.c_double),
                              _p(a, C.c_double), C.c_int(a.shape[0]), C.c_int(n_sub),
                              C.c_uint64(t0), None if pen is None else _p(pen, C.c_double),
                              C.c_double(beta or 0.0))
        if rc != 0:
            raise ValueError("or_rollout rejected its arguments")
        return s, pen

    def rollout_vjp(self, state0, actions, n_sub, t0, gstate, gpen=None, beta=None):
        """Reverse pass of rollout: returns (dL/d state0 [Q][27],
        dL/d actions [n_calls][Q][4], dL/d params [Q][6])."""
        s0 = np.ascontiguousarray(state0, dtype=np.float64)
        a = np.ascontiguousarray(actions, dtype=np.float64)
        g = np.array(gstate, dtype=np.float64, order="C", copy=True)
        gp = None if gpen is None else np.ascontiguousarray(gpen, dtype=np.float64)
        gact = np.zeros_like(a)
        gpar = np.zeros((self.Q, 6))
        rc = lib().or_rollout_vjp(C.byref(self.desc), _p(self.params, C.c_double),
                                  _p(s0, C.c_double), _p(a, C.c_double), C.c_int(a.shape[0]),
                                  C.c_int(n_sub), C.c_uint64(t0), _p(g, C.c_double),
                                  None if gp is None else _p(gp, C.c_double),
                                  C.c_double(beta or 0.0), _p(gact, C.c_double),
                                  _p(gpar, C.c_double))
        if rc != 0:
            raise ValueError("or_rollout_vjp rejected its arguments")
        return g, gact, gpar

    def observe_noise(self, obs, t: int):
        """Sensor noise added to a copy of obs (as or_observe returns it)."""
        o = np.array(obs, dtype=np.float64, order="C", copy=True)
        if lib().or_observe_noise(C.byref(self.desc), _p(o, C.c_double), C.c_uint64(t)) != 0:
            raise ValueError("or_observe_noise rejected its arguments")
        return o

    def reward(self, s0, s1, events, goals, obs, weights):
        """Per-quad reward of one call (see or_reward)."""
        a = np.ascontiguousarray(s0, dtype=np.float64)
        b = np.ascontiguousarray(s1, dtype=np.float64)
        ev = np.ascontiguousarray(events, dtype=np.uint32)
        g = np.ascontiguousarray(goals, dtype=np.float64)
        o = np.ascontiguousarray(obs, dtype=np.float64)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        assert w.shape == (15,)
        r = np.zeros(self.Q)
        if lib().or_reward(C.byref(self.desc), _p(self.params, C.c_double), _p(a, C.c_double),
                           _p(b, C.c_double), _p(ev, C.c_uint32), _p(g, C.c_double),
                           _p(o, C.c_double), _p(w, C.c_double), _p(r, C.c_double)) != 0:
            raise ValueError("or_reward rejected its arguments")
        return r

    def with_params(self, params) -> "Oracle":
        """Same environments and constants, other per-quad parameters."""
        o = Oracle.__new__(Oracle)
        o.__dict__.update(self.__dict__)
        o.params = np.ascontiguousarray(params, dtype=np.float64)
        return o

    def observe(self, state, goals):
        """Returns (obs [Q][18+6K] f64, neighbour local indices [Q][K] i32)."""
        s = np.ascontiguousarray(state, dtype=np.float64)
        g = np.ascontiguousarray(goals, dtype=np.float64)
        obs = np.zeros((self.Q, 18 + 6 * self.K))
        nbr = np.full((self.Q, max(self.K, 1)), -1, dtype=np.int32)
        rc = lib().or_observe(C.byref(self.desc), _p(s, C.c_double),
                              _p(g, C.c_double), _p(obs, C.c_double),
                              _p(nbr, C.c_int32))
        if rc != 0:
            raise ValueError("or_observe rejected its arguments")
        return obs, nbr[:, :self.K]


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def normal4(seed: int, quad: int, t: int, stream: int, draw: int):
    z = (C.c_double * 4)()
    lib().or_normal4(C.c_uint64(seed), C.c_uint32(quad), C.c_uint64(t),
                     C.c_uint32(stream), C.c_uint32(draw), z)
    return np.array(list(z))


def noise_batch(seed: int, stream: int, draw: int, t: int, quad0: int, n: int):
    """(words [n][4] uint32, normals [n][4] f64) of the generator for quads
    quad0 .. quad0 + n - 1 at substep t (see or_noise_batch)."""
    words = np.zeros((n, 4), dtype=np.uint32)
    normals = np.zeros((n, 4))
    rc = lib().or_noise_batch(C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), C.c_uint32(stream),
                              C.c_uint32(draw), C.c_uint64(t), C.c_uint32(quad0), C.c_int(n),
                              _p(words, C.c_uint32), _p(normals, C.c_double))
    if rc != 0:
        raise ValueError("or_noise_batch rejected its arguments")
    return words, normals


def uniform_from_u32(r: int) -> float:
    return float(lib().or_uniform_from_u32(C.c_uint32(r)))


def flag_values():
    o = (C.c_uint32 * 8)()
    lib().or_flag_values(o)
    return [int(v) for v in o]
