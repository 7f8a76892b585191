"""Python binding of the C ABI in include/quadswarm.h (ctypes).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of ``libquadswarm.so``.  PyTorch provides device memory and the
current stream; nothing here computes on tensors.  If the library is not
built, :func:`lib` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libquadswarm.so")

QS_OK = 0
ERRORS = {-1: "QS_ERR_NULL", -2: "QS_ERR_INVALID", -3: "QS_ERR_ENV_SIZE", -4: "QS_ERR_HIP",
          -5: "QS_ERR_NONFINITE", -6: "QS_ERR_NOMEM", -7: "QS_ERR_ALIGN", -8: "QS_ERR_UNSUPPORTED",
          -9: "QS_ERR_TOO_LARGE"}

# every entry point of include/quadswarm.h
EXPORTS = ("qs_create", "qs_destroy", "qs_sizes", "qs_substep_index", "qs_step", "qs_observe",
           "qs_step_observe", "qs_get_state", "qs_set_state", "qs_record_contacts",
           "qs_debug_contacts", "qs_sync", "qs_rollout", "qs_rollout_backward",
           "qs_step_backward", "qs_step_backward_noalloc", "qs_set_graph_mode", "qs_set_launch",
           "qs_autotune", "qs_set_partner_chunks", "qs_launch_plan", "qs_set_reward_weights", "qs_step_observe_reward", "qs_set_params",
           "qs_debug_philox", "qs_error_string")


class QuadSwarmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().qs_error_string(code).decode()
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({msg})")


class qs_desc(C.Structure):
    _fields_ = [
        ("n_envs", C.c_int32), ("env_offsets", C.POINTER(C.c_int32)),
        ("dt", C.c_float), ("gravity", C.c_float), ("arm_length", C.c_float),
        ("k_tau", C.c_float), ("drag_coef", C.c_float), ("floor_mu", C.c_float),
        ("motor_noise_decay", C.c_float), ("motor_noise_std", C.c_float),
        ("room_min", C.c_float * 3), ("room_max", C.c_float * 3),
        ("wall_restitution", C.c_float),
        ("col_dist", C.c_float), ("col_decay", C.c_float),
        ("col_noise_v", C.c_float), ("col_noise_w", C.c_float),
        ("k_neighbors", C.c_int32), ("flags", C.c_uint32), ("seed", C.c_uint64),
        ("dw_k1", C.c_float), ("dw_k2", C.c_float), ("dw_b1", C.c_float),
        ("dw_radius", C.c_float), ("dw_height", C.c_float),
        ("dw_noise_a", C.c_float), ("dw_noise_w", C.c_float),
        ("sn_x", C.c_float), ("sn_v", C.c_float), ("sn_w", C.c_float),
    ]


_lib = None


_F32 = None


def _f32():
    global _F32
    if _F32 is None:
        import torch
        _F32 = torch.float32
    return _F32


def lib() -> C.CDLL:
    """Load libquadswarm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2306_09537_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
        L.qs_create.argtypes = [C.POINTER(qs_desc), vp, vp, C.POINTER(vp)]
        L.qs_destroy.argtypes = [vp]
        L.qs_sizes.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.qs_step.argtypes = [vp, vp, i32, vp]
        L.qs_observe.argtypes = [vp, vp, vp, vp]
        L.qs_step_observe.argtypes = [vp, vp, i32, vp, vp, vp]
        L.qs_step_observe_reward.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.qs_set_reward_weights.argtypes = [vp, vp]
        L.qs_get_state.argtypes = [vp, vp, C.POINTER(u64), vp]
        L.qs_set_state.argtypes = [vp, vp, u64, vp, vp]
        L.qs_set_params.argtypes = [vp, vp, vp, vp]
        u32 = C.c_uint32
        L.qs_debug_philox.argtypes = [u64, u32, u32, u64, u32, i32, vp, vp, vp]
        L.qs_record_contacts.argtypes = [vp, i32]
        L.qs_debug_contacts.argtypes = [vp, vp, vp]
        L.qs_sync.argtypes = [vp, vp]
        L.qs_substep_index.argtypes = [vp, C.POINTER(u64)]
        f32 = C.c_float
        L.qs_rollout.argtypes = [vp, vp, i32, i32, i32, vp, vp, f32, vp]
        L.qs_rollout_backward.argtypes = [vp, vp, i32, i32, i32, vp, u64, vp, vp, f32, vp, vp, vp]
        L.qs_step_backward.argtypes = [vp, vp, vp, i32, u64, vp, vp, vp, vp, vp]
        L.qs_step_backward_noalloc.argtypes = [vp, vp, vp, i32, u64, vp, vp, vp, vp, vp]
        L.qs_set_graph_mode.argtypes = [vp, i32, vp]
        L.qs_autotune.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.qs_set_launch.argtypes = [vp, i32, i32]
        L.qs_set_partner_chunks.argtypes = [vp, C.c_uint32]
        L.qs_launch_plan.argtypes = [vp, vp, C.POINTER(i32)]
        L.qs_error_string.argtypes = [C.c_int]
        L.qs_error_string.restype = C.c_char_p
        for name in EXPORTS:
            if name != "qs_error_string":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != QS_OK:
        raise QuadSwarmError(rc, where)


def make_desc(env_offsets: np.ndarray, consts: dict, k_neighbors: int, flags: int,
              seed: int) -> qs_desc:
    d = qs_desc()
    d.n_envs = int(env_offsets.shape[0] - 1)
    d.env_offsets = env_offsets.ctypes.data_as(C.POINTER(C.c_int32))
    for k in ("dt", "gravity", "arm_length", "k_tau", "drag_coef", "floor_mu",
              "motor_noise_decay", "motor_noise_std", "wall_restitution", "col_dist",
              "col_decay", "col_noise_v", "col_noise_w"):
        setattr(d, k, float(consts[k]))
    d.room_min = (C.c_float * 3)(*[float(v) for v in consts["room_min"]])
    d.room_max = (C.c_float * 3)(*[float(v) for v in consts["room_max"]])
    d.k_neighbors = int(k_neighbors)
    d.flags = int(flags)
    d.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    for k in ("dw_k1", "dw_k2", "dw_b1", "dw_radius", "dw_height", "dw_noise_a", "dw_noise_w",
              "sn_x", "sn_v", "sn_w"):
        setattr(d, k, float(consts.get(k, 0.0)))
    return d


def _ptr(t) -> int:
    return int(t.data_ptr())


_RAW_STREAM = None


def _stream(device_index=None):
    """The current HIP stream of the device, as the C ABI's void*."""
    global _RAW_STREAM
    if _RAW_STREAM is None:
        import torch
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        # the raw getter builds no Stream object: a few microseconds less per call
        _RAW_STREAM = raw if raw is not None else (
            lambda i: torch.cuda.current_stream(i).cuda_stream)
    if device_index is None:
        import torch
        device_index = torch.cuda.current_device()
    return _RAW_STREAM(device_index)


class QuadSwarm:
    """One handle: E environments of swarms, Q quads, on the current device."""

    def __init__(self, env_offsets, consts: dict, params, state0, k_neighbors: int,
                 flags: int, seed: int):
        import torch
        self._offs = np.ascontiguousarray(env_offsets, dtype=np.int32)
        p = np.ascontiguousarray(params, dtype=np.float32)
        s0 = np.ascontiguousarray(state0, dtype=np.float32)
        desc = make_desc(self._offs, consts, k_neighbors, flags, seed)
        h = C.c_void_p()
        _check(lib().qs_create(C.byref(desc), p.ctypes.data, s0.ctypes.data, C.byref(h)),
               "qs_create")
        self._h = h
        q, e, od = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().qs_sizes(h, C.byref(q), C.byref(e), C.byref(od)), "qs_sizes")
        self.n_quads, self.n_envs, self.obs_dim = q.value, e.value, od.value
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._di = self.device.index
        # per-call constants of the stepping calls (their host time has to
        # stay below the kernel's)
        L = lib()
        self._f_step, self._f_observe = L.qs_step, L.qs_observe
        self._f_step_observe, self._f_step_observe_reward = L.qs_step_observe, L.qs_step_observe_reward
        Q = self.n_quads
        self._s_act, self._s_goal, self._s_obs, self._s_q = (Q, 4), (Q, 3), (Q, self.obs_dim), (Q,)

    @classmethod
    def from_workload(cls, w: "W.Workload") -> "QuadSwarm":
        return cls(w.env_offsets, w.consts, w.params, w.state0, w.k_neighbors, w.flags,
                   w.rng_key)

    # -- helpers -----------------------------------------------------------
    def _dev(self, t, shape, dtype=None):
        """t must be a contiguous tensor of this shape and dtype (float32 by
        default) on the handle's GPU.  Kept cheap: it runs on every call,
        and the host time of a call must stay below the kernel's.  (Buffer
        overlaps are refused by the library itself.)"""
        try:
            ok = (t.get_device() == self._di and t.dtype is (dtype or _f32())
                  and t.size() == shape and t.is_contiguous())
        except AttributeError:
            ok = False
        if not ok:
            raise ValueError(f"expected a contiguous {dtype or _f32()} tensor of shape "
                             f"{tuple(shape)} on cuda:{self._di}")
        return t

    # -- API ---------------------------------------------------------------
    def step(self, actions, n_substeps: int = 1) -> None:
        self._dev(actions, self._s_act)
        _check(self._f_step(self._h, actions.data_ptr(), int(n_substeps), _stream(self._di)),
               "qs_step")

    def _out_obs(self, out):
        if out is None:
            import torch
            out = torch.empty(self._s_obs, device=self.device)
        return self._dev(out, self._s_obs)

    def observe(self, goals, out=None):
        self._dev(goals, self._s_goal)
        o = self._out_obs(out)
        _check(self._f_observe(self._h, goals.data_ptr(), o.data_ptr(), _stream(self._di)),
               "qs_observe")
        return o

    def step_observe(self, actions, n_substeps: int, goals, out=None):
        self._dev(actions, self._s_act)
        self._dev(goals, self._s_goal)
        o = self._out_obs(out)
        _check(self._f_step_observe(self._h, actions.data_ptr(), int(n_substeps),
                                    goals.data_ptr(), o.data_ptr(), _stream(self._di)),
               "qs_step_observe")
        return o

    def set_reward_weights(self, weights) -> None:
        """The 15 reward weights (alpha_pos ... alpha_prox, d_prox)."""
        w = np.ascontiguousarray(weights, dtype=np.float32)
        if w.shape != (15,):
            raise ValueError("reward weights: expected 15 values")
        _check(lib().qs_set_reward_weights(self._h, w.ctypes.data), "qs_set_reward_weights")

    def step_observe_reward(self, actions, n_substeps: int, goals, out=None, reward=None):
        """step_observe that also returns each quad's reward of the call."""
        self._dev(actions, self._s_act)
        self._dev(goals, self._s_goal)
        o = self._out_obs(out)
        if reward is None:
            import torch
            reward = torch.empty(self._s_q, device=self.device)
        self._dev(reward, self._s_q)
        _check(self._f_step_observe_reward(self._h, actions.data_ptr(), int(n_substeps),
                                           goals.data_ptr(), o.data_ptr(), reward.data_ptr(),
                                           _stream(self._di)), "qs_step_observe_reward")
        return o, reward

    def get_state(self, out=None):
        import torch
        o = out if out is not None else torch.empty((self.n_quads, 27), device=self.device)
        self._dev(o, (self.n_quads, 27))
        t = C.c_uint64()
        _check(lib().qs_get_state(self._h, _ptr(o), C.byref(t), _stream(self._di)), "qs_get_state")
        return o, int(t.value)

    def set_state(self, state, substep: int, env_mask=None) -> None:
        import torch
        s = self._dev(state, (self.n_quads, 27))
        m = None
        if env_mask is not None:
            m = self._dev(env_mask, (self.n_envs,), torch.uint8)
        _check(lib().qs_set_state(self._h, _ptr(s), C.c_uint64(int(substep)),
                                  None if m is None else _ptr(m), _stream(self._di)), "qs_set_state")

    def set_params(self, params, env_mask=None) -> None:
        """qs_set_params: per-quad (mass, ixx, iyy, izz, thrust_to_weight,
        tau_m) [Q][6] on the handle's device; f_max and alpha_lag are
        re-derived on the device."""
        import torch
        p = self._dev(params, (self.n_quads, 6))
        m = None
        if env_mask is not None:
            m = self._dev(env_mask, (self.n_envs,), torch.uint8)
        _check(lib().qs_set_params(self._h, _ptr(p), None if m is None else _ptr(m),
                                   _stream(self._di)), "qs_set_params")

    def record_contacts(self, enable: bool = True) -> None:
        _check(lib().qs_record_contacts(self._h, 1 if enable else 0), "qs_record_contacts")

    def debug_contacts(self):
        import torch
        o = torch.empty(self.n_quads, dtype=torch.int64, device=self.device)
        _check(lib().qs_debug_contacts(self._h, _ptr(o), _stream(self._di)), "qs_debug_contacts")
        return o

    @property
    def substep(self) -> int:
        t = C.c_uint64()
        _check(lib().qs_substep_index(self._h, C.byref(t)), "qs_substep_index")
        return int(t.value)

    def rollout(self, actions, n_substeps: int, ckpt_every: int = 0, ckpt=None, penalty=None,
                beta: float = 0.0) -> None:
        """qs_rollout over actions [n_calls][Q][4]."""
        a = actions
        n_calls = a.shape[0]
        self._dev(a, (n_calls, self.n_quads, 4))
        if ckpt is not None:
            if ckpt_every <= 0:
                raise ValueError("checkpoints need ckpt_every >= 1")
            n_ck = (n_calls + ckpt_every - 1) // ckpt_every
            self._dev(ckpt, (n_ck, 27, self.n_quads))
        if penalty is not None:
            self._dev(penalty, (self.n_quads,))
        _check(lib().qs_rollout(self._h, _ptr(a), n_calls, int(n_substeps), int(ckpt_every),
                                None if ckpt is None else _ptr(ckpt),
                                None if penalty is None else _ptr(penalty), float(beta),
                                _stream(self._di)), "qs_rollout")

    def rollout_backward(self, actions, n_substeps: int, ckpt_every: int, ckpt,
                         substep_index0: int, gstate, gpenalty, beta: float, gactions,
                         gparams) -> None:
        """qs_rollout_backward (gstate is overwritten with dL/d initial state)."""
        n_calls = actions.shape[0]
        if ckpt_every <= 0:
            raise ValueError("the backward pass needs ckpt_every >= 1")
        n_ck = (n_calls + ckpt_every - 1) // ckpt_every
        self._dev(actions, (n_calls, self.n_quads, 4))
        self._dev(ckpt, (n_ck, 27, self.n_quads))
        self._dev(gactions, (n_calls, self.n_quads, 4))
        self._dev(gstate, (self.n_quads, 27))
        self._dev(gparams, (self.n_quads, 6))
        if gpenalty is not None:
            self._dev(gpenalty, (self.n_quads,))
        _check(lib().qs_rollout_backward(
            self._h, _ptr(actions), n_calls, int(n_substeps), int(ckpt_every), _ptr(ckpt),
            C.c_uint64(int(substep_index0)), _ptr(gstate),
            None if gpenalty is None else _ptr(gpenalty), float(beta), _ptr(gactions),
            _ptr(gparams), _stream(self._di)), "qs_rollout_backward")

    def step_backward(self, state_in, actions, n_substeps: int, substep_index: int,
                      gstate_out, gstate_in, gactions, gparams) -> None:
        Q = self.n_quads
        for tns, shp in ((state_in, (Q, 27)), (actions, (Q, 4)), (gstate_out, (Q, 27)),
                         (gstate_in, (Q, 27)), (gactions, (Q, 4)), (gparams, (Q, 6))):
            self._dev(tns, shp)
        _check(lib().qs_step_backward(self._h, _ptr(state_in), _ptr(actions), int(n_substeps),
                                      C.c_uint64(int(substep_index)), _ptr(gstate_out),
                                      _ptr(gstate_in), _ptr(gactions), _ptr(gparams),
                                      _stream(self._di)), "qs_step_backward")

    def step_backward_noalloc(self, state_in, actions, n_substeps: int, substep_index: int,
                              gstate_out, gstate_in, gactions, gparams) -> None:
        """qs_step_backward_noalloc: as step_backward, with the library's
        fixed per-device scratch instead of any device allocation."""
        Q = self.n_quads
        for tns, shp in ((state_in, (Q, 27)), (actions, (Q, 4)), (gstate_out, (Q, 27)),
                         (gstate_in, (Q, 27)), (gactions, (Q, 4)), (gparams, (Q, 6))):
            self._dev(tns, shp)
        _check(lib().qs_step_backward_noalloc(
            self._h, _ptr(state_in), _ptr(actions), int(n_substeps),
            C.c_uint64(int(substep_index)), _ptr(gstate_out), _ptr(gstate_in), _ptr(gactions),
            _ptr(gparams), _stream(self._di)), "qs_step_backward_noalloc")

    def set_graph_mode(self, enable: bool = True) -> None:
        _check(lib().qs_set_graph_mode(self._h, 1 if enable else 0, _stream(self._di)),
               "qs_set_graph_mode")

    def set_launch(self, block: int, grid: int = 0) -> None:
        _check(lib().qs_set_launch(self._h, int(block), int(grid)), "qs_set_launch")

    def autotune(self, actions, n_substeps: int, goals=None, out=None) -> dict:
        """qs_autotune: returns the chosen (block, grid, bucketed) and the
        per-slot-size plan (launch_plan)."""
        self._dev(actions, (self.n_quads, 4))
        ch = (C.c_int32 * 3)()
        _check(lib().qs_autotune(self._h, _ptr(actions), int(n_substeps),
                                 None if goals is None else _ptr(goals),
                                 None if out is None else _ptr(out), ch, _stream(self._di)),
               "qs_autotune")
        return {"block": ch[0], "grid": ch[1], "bucketed": bool(ch[2]),
                "slots": self.launch_plan()}

    def set_partner_chunks(self, slots) -> None:
        """qs_set_partner_chunks: the slot sizes (16, 32) whose items take
        the in-swarm partners in chunks of four in the bucketed form."""
        mask = 0
        for n in slots:
            mask |= 1 << (int(n).bit_length() - 1)
        _check(lib().qs_set_partner_chunks(self._h, mask), "qs_set_partner_chunks")

    def launch_plan(self) -> list:
        """qs_launch_plan: per slot size, its swarms, whether its items take
        the chunked body, and the autotuner's times (ns) for its items with
        the one-partner and with the chunked body."""
        buf = (C.c_int32 * 35)()
        n = C.c_int32()
        _check(lib().qs_launch_plan(self._h, buf, C.byref(n)), "qs_launch_plan")
        return [{"slot": buf[5 * r], "swarms": buf[5 * r + 1], "chunked": bool(buf[5 * r + 2]),
                 "ns_one": buf[5 * r + 3], "ns_chunked": buf[5 * r + 4]}
                for r in range(n.value)]

    def sync(self) -> None:
        _check(lib().qs_sync(self._h, _stream(self._di)), "qs_sync")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().qs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def debug_philox(seed: int, noise_stream: int, draw: int, substep_index: int, quad0: int,
                 n: int, with_normals: bool = True, device=None):
    """qs_debug_philox: the library's generator words [n][4] (int32 tensor
    holding the uint32 bits) and, optionally, its N(0,1) draws [n][4]."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    words = torch.empty((n, 4), dtype=torch.int32, device=dev)
    normals = torch.empty((n, 4), dtype=torch.float32, device=dev) if with_normals else None
    _check(lib().qs_debug_philox(C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(noise_stream),
                                 int(draw), C.c_uint64(int(substep_index)), int(quad0), int(n),
                                 _ptr(words), None if normals is None else _ptr(normals),
                                 _stream(dev.index)), "qs_debug_philox")
    return words, normals


def _make_rollout_fn():
    import torch

    class RolloutFn(torch.autograd.Function):
        """Differentiable rollout through the HIP forward and adjoint kernels.

        forward(state0 [Q][27], actions [T][Q][4], params [Q][6], sim,
        n_substeps, ckpt_every, beta) -> (final state [Q][27], penalty [Q]).
        ``params`` (mass, ixx, iyy, izz, thrust_to_weight, tau_m per quad)
        are loaded into the handle (qs_set_params) before the rollout, so the
        simulation runs with them and dL/d params belongs to them; the handle
        keeps them afterwards.  The forward keeps ceil(T / ckpt_every)
        checkpoints; the backward recomputes each segment from its
        checkpoint.
        """

        @staticmethod
        def forward(ctx, state0, actions, params, sim, n_substeps, ckpt_every, beta):
            T = actions.shape[0]
            t0 = sim.substep
            sim.set_params(params.detach().contiguous())
            sim.set_state(state0.detach().contiguous(), t0)
            n_ck = (T + ckpt_every - 1) // ckpt_every
            ckpt = torch.empty((n_ck, 27, sim.n_quads), device=state0.device)
            pen = torch.zeros(sim.n_quads, device=state0.device)
            acts = actions.detach().contiguous()
            sim.rollout(acts, n_substeps, ckpt_every, ckpt, pen if beta > 0 else None, beta)
            sT, _ = sim.get_state()
            ctx.save_for_backward(acts, ckpt)
            ctx.sim, ctx.nsub, ctx.ce, ctx.beta, ctx.t0 = sim, n_substeps, ckpt_every, beta, t0
            return sT, pen

        @staticmethod
        def backward(ctx, g_state, g_pen):
            acts, ckpt = ctx.saved_tensors
            sim = ctx.sim
            Q = sim.n_quads
            gstate = (g_state.contiguous().clone() if g_state is not None
                      else torch.zeros((Q, 27), device=acts.device))
            gpen = None
            if g_pen is not None and ctx.beta > 0:
                gpen = g_pen.contiguous()
            gact = torch.empty_like(acts)
            gpar = torch.zeros((Q, 6), device=acts.device)
            sim.rollout_backward(acts, ctx.nsub, ctx.ce, ckpt, ctx.t0, gstate, gpen, ctx.beta,
                                 gact, gpar)
            return gstate, gact, gpar, None, None, None, None

    return RolloutFn


_ROLLOUT_FN = None


def rollout(sim: QuadSwarm, state0, actions, params, n_substeps: int = 1, ckpt_every: int = 20,
            beta: float = 100.0):
    """Differentiable rollout: returns (final state, per-quad penalty)."""
    global _ROLLOUT_FN
    if _ROLLOUT_FN is None:
        _ROLLOUT_FN = _make_rollout_fn()
    return _ROLLOUT_FN.apply(state0, actions, params, sim, n_substeps, ckpt_every, beta)
