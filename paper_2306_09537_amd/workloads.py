"""Seeded synthetic workloads for the batched quadrotor-swarm step.

This module only *draws inputs*: per-quad physical parameters (the domain
randomisation named in §I and §III-A), initial states, goals and per-step
action sequences, plus the global constants and physics switches of each
workload.  It contains none of the simulator's arithmetic.  Both the FP64
oracle (test infrastructure) and the GPU library receive exactly what this
module returns, rounded once to float32, so the two start from identical
inputs.

Workloads (all quads advance with dt = 5 ms, the 200 Hz simulation rate of §IV):

  plain   64 envs x 1 quad, nominal Crazyflie parameters, no room/floor/pairs
  swarm8  4096 envs x 8 quads, +-20 % mass/inertia/thrust-to-weight, +-30 %
          motor time constant, motor noise sigma 0.05, 10x10x10 m room with
          walls/ceiling and floor, pairwise collisions at 0.1 m, K = 6
  uneven  16384 envs with swarm sizes drawn from {1,2,4,8,16,32}, physics as swarm8
  diff    1024 envs x 8 quads, physics as swarm8
  scale32 32768 envs x 32 quads, physics as swarm8
  scale1  1,048,576 envs x 1 quad, physics as swarm8 without pairs, K = 0

Every generator takes ``n_envs`` so tests can run the same structure smaller.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# Interface constants shared by value with the C ABI (include/quadswarm.h) and
# the oracle; tests check that the three agree.
# ---------------------------------------------------------------------------
QS_ROOM = 1            # walls and ceiling of the room bounce the quad
QS_FLOOR = 2           # floor model: hit, rest, friction, take-off
QS_COLLIDE = 4         # in-env pairwise collision detection and response
QS_MOTOR_NOISE = 8     # AR(1) motor-noise process
QS_APPROACH_ONLY = 16  # pair response only while the pair is approaching
QS_ACT_UNIT = 32       # action read as normalised thrust in [0,1] (else [-1,1])
QS_DOWNWASH = 64       # downwash of upper quads on lower ones (§III-B.4)
QS_SENSOR_NOISE = 128  # noise on the observed position, velocity, body rate (§III-C)

STATE_DIM = 27         # x3 v3 R9 (row-major) w3 u4 eps4 floor1
PARAM_DIM = 6          # mass, ixx, iyy, izz, thrust_to_weight, motor_tau
ACT_DIM = 4
GOAL_DIM = 3
SX, SV, SR, SW, SU, SE, SF = 0, 3, 6, 15, 18, 22, 26


def obs_dim(k: int) -> int:
    return 18 + 6 * k


# Nominal Crazyflie-class constants of the workloads.
NOMINAL = dict(mass=0.028, ixx=1.66e-5, iyy=1.66e-5, izz=2.93e-5,
               thrust_to_weight=2.0, motor_tau=0.015)

BASE_CONSTS = dict(
    dt=0.005, gravity=9.81, arm_length=0.046, k_tau=0.006, drag_coef=0.0,
    floor_mu=0.6, motor_noise_decay=0.9, motor_noise_std=0.05,
    room_min=(-5.0, -5.0, 0.0), room_max=(5.0, 5.0, 10.0),
    wall_restitution=1.0, col_dist=0.1, col_decay=1.0,
    col_noise_v=0.0, col_noise_w=0.0,
    # downwash: -k1 (k2 dz + b1) e_z, i.e. 2 m/s^2 decaying linearly to zero
    # at 0.5 m of vertical separation, within 0.1 m of horizontal offset
    dw_k1=2.0, dw_k2=-2.0, dw_b1=1.0, dw_radius=0.1, dw_height=0.5,
    dw_noise_a=0.0, dw_noise_w=0.0,
    # observation sensor noise: U(-5e-3, 5e-3) m, U(-1e-2, 1e-2) m/s, N(0, 1.75e-4^2) rad/s
    sn_x=5e-3, sn_v=1e-2, sn_w=1.75e-4,
)

# Reward weights (alpha_pos, _vel, _ori, _spin, _act, _dact, _rot, _yaw,
# _floor_hit, _on_floor, _wall, _ceiling, _quad, _prox, d_prox); the paper
# names the terms but not their weights.
REWARD_WEIGHTS = (-1.0, -0.1, 0.2, -0.05, -0.05, -0.1, 0.0, 0.0,
                  -5.0, -1.0, -2.0, -2.0, -5.0, -1.0, 0.5)

SWARM_FLAGS = QS_ROOM | QS_FLOOR | QS_COLLIDE | QS_MOTOR_NOISE | QS_APPROACH_ONLY


@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    env_sizes: np.ndarray        # int32 [E]
    env_offsets: np.ndarray      # int32 [E+1], CSR
    consts: dict
    k_neighbors: int
    flags: int
    rng_key: int                 # uint64 key of the method's counter-based noise
    params: np.ndarray           # float32 [Q][6]
    state0: np.ndarray           # float32 [Q][27]
    goals: np.ndarray            # float32 [Q][3]
    substeps: int                # rollout length of the workload
    act_low: float = 0.0
    act_high: float = 1.0

    @property
    def n_envs(self) -> int:
        return int(self.env_sizes.shape[0])

    @property
    def n_quads(self) -> int:
        return int(self.env_offsets[-1])

    @property
    def obs_dim(self) -> int:
        return obs_dim(self.k_neighbors)

    def actions(self, step: int) -> np.ndarray:
        """Actions of one control call, float32 [Q][4], U[act_low, act_high]."""
        rng = np.random.Generator(np.random.PCG64([self.seed, 0xAC7, step]))
        a = rng.uniform(self.act_low, self.act_high, size=(self.n_quads, ACT_DIM))
        return a.astype(np.float32)

    def action_sequence(self, n_steps: int) -> np.ndarray:
        """float32 [n_steps][Q][4], one independent draw per call."""
        rng = np.random.Generator(np.random.PCG64([self.seed, 0xAC8, n_steps]))
        a = rng.random(size=(n_steps, self.n_quads, ACT_DIM), dtype=np.float32)
        return (self.act_low + (self.act_high - self.act_low) * a).astype(np.float32)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _rot_axis_angle(axis: np.ndarray, ang: np.ndarray) -> np.ndarray:
    """Rotation matrices [N][3][3] about unit axes [N][3] by angles [N]."""
    c, s = np.cos(ang), np.sin(ang)
    x, y, z = axis[:, 0], axis[:, 1], axis[:, 2]
    C = 1.0 - c
    R = np.empty((axis.shape[0], 3, 3))
    R[:, 0, 0] = c + x * x * C
    R[:, 0, 1] = x * y * C - z * s
    R[:, 0, 2] = x * z * C + y * s
    R[:, 1, 0] = y * x * C + z * s
    R[:, 1, 1] = c + y * y * C
    R[:, 1, 2] = y * z * C - x * s
    R[:, 2, 0] = z * x * C - y * s
    R[:, 2, 1] = z * y * C + x * s
    R[:, 2, 2] = c + z * z * C
    return R


def draw_params(rng: np.random.Generator, q: int, randomise: bool) -> np.ndarray:
    p = np.empty((q, PARAM_DIM))
    names = ("mass", "ixx", "iyy", "izz", "thrust_to_weight", "motor_tau")
    for k, nm in enumerate(names):
        p[:, k] = NOMINAL[nm]
    if randomise:
        for k in range(5):
            p[:, k] *= rng.uniform(0.8, 1.2, size=q)
        p[:, 5] *= rng.uniform(0.7, 1.3, size=q)
    return p


def draw_state0(rng: np.random.Generator, params: np.ndarray) -> np.ndarray:
    """Initial states: position U([-2,2]^2 x [0.5,2.5]) m, velocity and body
    rate N(0, 0.5^2) per component, attitude within 30 deg of upright with a
    uniform yaw, motors at the hover command, zero motor noise, airborne."""
    q = params.shape[0]
    s = np.zeros((q, STATE_DIM))
    s[:, 0:2] = rng.uniform(-2.0, 2.0, size=(q, 2))
    s[:, 2] = rng.uniform(0.5, 2.5, size=q)
    s[:, SV:SV + 3] = rng.normal(0.0, 0.5, size=(q, 3))
    phi = rng.uniform(0.0, 2 * math.pi, size=q)
    psi = rng.uniform(0.0, 2 * math.pi, size=q)
    cos_t = rng.uniform(math.cos(math.radians(30.0)), 1.0, size=q)
    theta = np.arccos(cos_t)
    tilt_axis = np.stack([np.cos(phi), np.sin(phi), np.zeros(q)], axis=1)
    z_axis = np.tile(np.array([0.0, 0.0, 1.0]), (q, 1))
    R = _rot_axis_angle(tilt_axis, theta) @ _rot_axis_angle(z_axis, psi)
    s[:, SR:SR + 9] = R.reshape(q, 9)
    s[:, SW:SW + 3] = rng.normal(0.0, 0.5, size=(q, 3))
    s[:, SU:SU + 4] = np.sqrt(1.0 / params[:, 4])[:, None]
    return s


def _finish(name, seed, sizes, consts, k, flags, randomise, substeps) -> Workload:
    rng = np.random.Generator(np.random.PCG64([seed, 0x5EED]))
    sizes = np.asarray(sizes, dtype=np.int32)
    offs = np.zeros(sizes.shape[0] + 1, dtype=np.int32)
    np.cumsum(sizes, out=offs[1:])
    q = int(offs[-1])
    params = draw_params(rng, q, randomise)
    state0 = draw_state0(rng, params)
    goals = np.empty((q, 3))
    goals[:, 0:2] = rng.uniform(-3.0, 3.0, size=(q, 2))
    goals[:, 2] = rng.uniform(1.0, 3.0, size=q)
    return Workload(
        name=name, seed=seed, env_sizes=sizes, env_offsets=offs,
        consts=dict(consts), k_neighbors=k, flags=flags,
        rng_key=(0x9E3779B97F4A7C15 * (seed + 1)) & 0xFFFFFFFFFFFFFFFF,
        params=params.astype(np.float32), state0=state0.astype(np.float32),
        goals=goals.astype(np.float32), substeps=substeps)


def plain(seed: int = 0, n_envs: int = 64, noise: bool = False) -> Workload:
    flags = QS_MOTOR_NOISE if noise else 0
    return _finish("plain_64x1", seed, [1] * n_envs, BASE_CONSTS, 0, flags,
                   randomise=False, substeps=1000)


def swarm8(seed: int = 0, n_envs: int = 4096) -> Workload:
    return _finish("swarm_4096x8", seed, [8] * n_envs, BASE_CONSTS, 6,
                   SWARM_FLAGS, randomise=True, substeps=1000)


def uneven(seed: int = 0, n_envs: int = 16384) -> Workload:
    rng = np.random.Generator(np.random.PCG64([seed, 0x517E]))
    sizes = rng.choice(np.array([1, 2, 4, 8, 16, 32]), size=n_envs)
    return _finish("uneven_16384", seed, sizes, BASE_CONSTS, 6, SWARM_FLAGS,
                   randomise=True, substeps=1000)


def diff(seed: int = 0, n_envs: int = 1024) -> Workload:
    return _finish("diff_1024x8", seed, [8] * n_envs, BASE_CONSTS, 6,
                   SWARM_FLAGS, randomise=True, substeps=200)


def scale32(seed: int = 0, n_envs: int = 32768) -> Workload:
    return _finish("scale_32768x32", seed, [32] * n_envs, BASE_CONSTS, 6,
                   SWARM_FLAGS, randomise=True, substeps=100)


def scale1(seed: int = 0, n_envs: int = 1048576) -> Workload:
    return _finish("scale_1048576x1", seed, [1] * n_envs, BASE_CONSTS, 0,
                   SWARM_FLAGS & ~QS_COLLIDE, randomise=True, substeps=100)


WORKLOADS = dict(plain=plain, swarm8=swarm8, uneven=uneven, diff=diff,
                 scale32=scale32, scale1=scale1)


def custom(sizes, *, seed: int = 0, k: int = 6, flags: int = SWARM_FLAGS,
           randomise: bool = True, name: str = "custom", **consts) -> Workload:
    """A workload with explicit swarm sizes and constant overrides."""
    c = dict(BASE_CONSTS)
    c.update(consts)
    return _finish(name, seed, sizes, c, k, flags, randomise, substeps=100)
