"""Throughput benchmark of the batched quadrotor-swarm step on one MI355X.

Default workload: 4096 environments x 8 quadrotors (32,768 quads), full
physics (motor lag and noise, walls, floor, in-env collisions) and the K = 6
nearest-neighbour observation, dt = 5 ms.  One timed "step" is one call of
the whole hot path over the batch: ``qs_step_observe`` with ``--nsub``
substeps (default 1: every row of the path, including the observation, runs
once per substep), on inputs already resident in HBM.  Rollouts are the
workload's 1000-substep episodes with a fresh action set per call; the
state is reset to the initial state between episodes outside the timed
region.

Prints one JSON line.  value = quad-steps/s (quads x substeps / s).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# VALU roofline: 256 CUs x 4 SIMDs at 2.4 GHz = 2457.6 G SIMD-cycles/s.  A
# kernel's VALU busy cycles come from its rocprofv3 counters with per-kind
# issue costs measured on the chip (calib/valu_probe): a wave64 FP32 add,
# multiply or FMA occupies a SIMD for 4 cycles, integer and bitwise
# instructions for 2 to 4, a transcendental 8 alone but it can overlap other
# VALU work.  Lower bound: 4 x (ADD + MUL + FMA) + 2 x every other
# non-transcendental VALU instruction; upper bound: 4 x SQ_ACTIVE_INST_VALU
# (one quad-cycle per instruction, two per transcendental).  The lower bound
# is reported as the fraction.
SIMD_GCYCLES_PER_S = 256 * 4 * 2.4
FP32_PEAK_TFLOPS = 157.3       # FP32 vector peak (packed FMA)
# committed counter summaries of the ten-substep form, per workload
VALU_PROFILES = {"swarm8": ("step_pipe_kernel_swarm4096x8_fused10.md", ""),
                 "scale32": ("scale_workloads.md", "scale32_")}
# ... and of the differentiable rollout and its backward pass
FWDBWD_PROFILES = {"diff_1024x8": ("rollout_reverse_diff1024x8.md", ""),
                   "scale_32768x32": ("scale_workloads.md", "scale32_")}
KERNEL_SOURCES = tuple(f"paper_2306_09537_amd/csrc/{f}" for f in
                       ("qs_device.h", "qs_kernels.h", "qs_rollout.h", "qs_adjoint.h"))
STATE_B, PARAM_B, ACT_B, GOAL_B = 108, 24, 16, 12


def algorithmic_bytes_per_quad(k: int, nsub: int, with_obs: bool = True) -> int:
    """Bytes one call must move per quad: state in and out, parameters,
    action, and (with the observation) goal and obs row."""
    b = 2 * STATE_B + PARAM_B + ACT_B
    if with_obs:
        b += GOAL_B + 4 * (18 + 6 * k)
    return b


def kernel_source_hash() -> str:
    import hashlib
    m = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_counter(profile: str, key: str):
    """A per-launch counter value ("key: value" line) from a committed
    rocprofv3 summary, or None if the kernel source changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
    except OSError:
        return None
    if kernel_source_hash() not in text:
        return None
    for line in text.splitlines():
        if line.startswith(key + ":"):
            return int(line.split(":")[1])
    return None


def measured_traffic(profile: str):
    """HBM bytes per launch from the committed counter summary."""
    return measured_counter(profile, "traffic_bytes_per_launch")


# committed counter summaries of the one-substep launch, per workload
TRAFFIC_PROFILES = {"swarm8": ("step_kernel_swarm4096x8_plain.md", "traffic_bytes_per_launch"),
                    "scale32": ("scale_workloads.md", "scale32_traffic_bytes_per_launch"),
                    "scale1": ("scale_workloads.md", "scale1_traffic_bytes_per_launch")}


def launch_traffic(workload: str, nsub: int):
    """Counter-measured HBM bytes of the timed launch, where committed (one
    substep per call) and taken on the current kernel sources."""
    if nsub != 1 or workload not in TRAFFIC_PROFILES:
        return None
    return measured_counter(*TRAFFIC_PROFILES[workload])


def alu_roofline(prof: str, key: str, ms: float):
    """ALU roofline of a kernel (or kernel sequence) from the committed
    counters under ``key``: VALU busy SIMD-cycles per second (lower bound)
    against the chip's SIMD-cycles per second, the upper-bound fraction,
    and FP32 FLOP/s against the vector peak.  None without counters."""
    lo = measured_counter(prof, key + "valu_busy_lo_cycles")
    hi = measured_counter(prof, key + "valu_busy_hi_cycles")
    flops = measured_counter(prof, key + "fp32_flops")
    if lo is None or hi is None or flops is None:
        return None
    s = ms * 1e-3
    ach = lo / s / 1e9
    tflops = flops / s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": SIMD_GCYCLES_PER_S,
            "unit": "G SIMD-cycles/s (VALU busy, lower bound)", "frac": ach / SIMD_GCYCLES_PER_S,
            "frac_upper": hi / s / 1e9 / SIMD_GCYCLES_PER_S, "traffic": None,
            "fp32_tflops": tflops, "fp32_frac_of_157_3": tflops / FP32_PEAK_TFLOPS,
            "valu_busy_cycles": [lo, hi], "fp32_flops": flops, "profile": prof}


def valu_roofline(workload: str, nsub: int, ms: float):
    """ALU roofline of the ten-substep launch of a workload."""
    if nsub != 10 or workload not in VALU_PROFILES:
        return None
    prof, pre = VALU_PROFILES[workload]
    return alu_roofline(prof, pre + "fused10_", ms)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="swarm8",
                    choices=["swarm8", "plain", "uneven", "diff", "scale32", "scale1"])
    ap.add_argument("--nsub", type=int, default=1, help="substeps per call")
    ap.add_argument("--extra-nsub", default="2,10",
                    help="also time these fused substep counts (comma list, '' for none)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fwdbwd", default="diff", help="workload of the fwd+bwd leg ('' to skip)")
    ap.add_argument("--fwdbwd-horizon", type=int, default=200)
    ap.add_argument("--batched", default="uneven", help="workload of the batched leg ('' to skip)")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only time the FP64 oracle on samples of every configuration "
                         "(host cores, no GPU) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (a kernel of "
                         "known traffic for scaling HBM counters) and exit")
    return ap.parse_args()


def time_calls(sim, w, acts, goals, obs, nsub, steps, warmup, torch, episode=1000):
    """Time ``steps`` calls of qs_step_observe with ``nsub`` substeps.

    Rollouts follow the workload's episodes: the state is reset to the
    initial state (untimed) whenever ``episode`` substeps have been taken;
    every call gets its own fresh action set (acts[i]).  Returns (ms per call
    from HIP events around the timed region on the launch stream -- the
    kernel is the only work on that stream, so this is its mean launch
    duration including dispatch gaps -- and host wall ms per call).
    """
    per_ep = max(1, episode // nsub)
    s0 = torch.from_numpy(w.state0).cuda()
    t_sub = [0]
    views = [acts[i] for i in range(acts.shape[0])]  # per-call action sets, sliced untimed

    def reset():
        sim.set_state(s0, t_sub[0])

    def call(i):
        sim.step_observe(views[i % len(views)], nsub, goals, obs)
        t_sub[0] += nsub

    reset()
    for i in range(warmup):
        if i and i % per_ep == 0:
            reset()
        call(i)
    sim.sync()
    total_ms, wall = 0.0, 0.0
    done = 0
    while done < steps:
        reset()
        n = min(per_ep, steps - done)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record()
        for i in range(n):
            call(done + i)
        end.record()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        total_ms += start.elapsed_time(end)
        done += n
    sim.sync()
    return total_ms / steps, wall * 1e3 / steps


def time_fwd_bwd(w, torch, horizon: int, nsub: int, ckpt_every: int, reps: int, beta=100.0):
    """Differentiable rollout of ``horizon`` calls (checkpoints every
    ``ckpt_every`` calls, smoothed collision penalty) and its reverse pass,
    each timed with HIP events on the launch stream; the state is reset to
    the initial state (untimed) before each repetition."""
    from paper_2306_09537_amd.quadswarm import QuadSwarm
    sim = QuadSwarm.from_workload(w)
    Q = w.n_quads
    acts = torch.from_numpy(w.action_sequence(horizon)).cuda()
    s0 = torch.from_numpy(w.state0).cuda()
    n_ck = (horizon + ckpt_every - 1) // ckpt_every
    ckpt = torch.empty((n_ck, 27, Q), device="cuda")
    pen = torch.zeros(Q, device="cuda")
    gs0 = torch.randn((Q, 27), device="cuda")
    gs0[:, 26] = 0
    gpen = torch.ones(Q, device="cuda")
    gstate = torch.empty_like(gs0)
    gact = torch.empty_like(acts)
    gpar = torch.zeros((Q, 6), device="cuda")
    fwd, bwd = [], []
    for r in range(reps + 1):
        t0 = r * horizon * nsub
        sim.set_state(s0, t0)
        gstate.copy_(gs0)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        sim.rollout(acts, nsub, ckpt_every, ckpt, pen, beta)
        e[1].record()
        sim.rollout_backward(acts, nsub, ckpt_every, ckpt, t0, gstate, gpen, beta, gact, gpar)
        e[2].record()
        torch.cuda.synchronize()
        if r:  # the first repetition warms up (scratch allocation)
            fwd.append(e[0].elapsed_time(e[1]))
            bwd.append(e[1].elapsed_time(e[2]))
    sim.sync()
    sim.close()
    f, b = float(np.median(fwd)), float(np.median(bwd))
    steps = Q * horizon * nsub
    # algorithmic bytes of the backward pass per quad-substep: tape write and
    # read (2 x 124: the state and the motor-noise draws), actions read twice
    # (2 x 16), action gradient (16); per
    # segment: its checkpoint and the parameters, read by the recompute
    # (108 + 24); once: adjoint in/out (216), parameters and their gradient
    # in the reverse sweep (32 + 48)
    seg = ckpt_every * nsub
    n_seg = (horizon + ckpt_every - 1) // ckpt_every
    bwd_bytes = Q * horizon * nsub * (248 + 32 + 16) + Q * n_seg * (108 + 24) + Q * (216 + 80)
    return dict(workload=w.name, quads=Q, horizon_substeps=horizon * nsub, ckpt_every=ckpt_every,
                value=steps / ((f + b) * 1e-3), unit="quad-steps/s (fwd+bwd)",
                fwd_ms=f, bwd_ms=b, fwd_value=steps / (f * 1e-3),
                bwd_roofline={"bound": "hbm", "achieved": bwd_bytes / (b * 1e-3) / 1e9,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": bwd_bytes / (b * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "traffic": fwdbwd_counter(w.name, horizon,
                                                        "backward_traffic_bytes"),
                              "bytes": bwd_bytes, "segment_substeps": seg},
                fwd_alu=fwdbwd_alu(w.name, horizon, "rollout_", f),
                bwd_alu=fwdbwd_alu(w.name, horizon, "backward_", b))


def fwdbwd_alu(name: str, horizon: int, part: str, ms: float):
    """ALU roofline of the rollout or of the backward pass (recompute and
    reverse sweeps together) at the horizon the counters were taken at."""
    if name not in FWDBWD_PROFILES:
        return None
    prof, pre = FWDBWD_PROFILES[name]
    if measured_counter(prof, pre + "fwdbwd_horizon") != horizon:
        return None
    return alu_roofline(prof, pre + part, ms)


def fwdbwd_counter(name: str, horizon: int, key: str):
    """A committed counter value of the fwd+bwd leg (e.g. the backward pass's
    HBM bytes), only at the horizon it was taken at."""
    if name not in FWDBWD_PROFILES:
        return None
    prof, pre = FWDBWD_PROFILES[name]
    if measured_counter(prof, pre + "fwdbwd_horizon") != horizon:
        return None
    return measured_counter(prof, pre + key)


def sticky_nonfinite(sim, torch) -> int:
    """Number of quads whose state is non-finite (the explicit integration of
    Euler's equation can diverge for a quad driven to very high spin rates);
    clears the handle's sticky error."""
    from paper_2306_09537_amd.quadswarm import QuadSwarmError
    try:
        sim.sync()
        return 0
    except QuadSwarmError:
        s, _ = sim.get_state()
        return int((~torch.isfinite(s).all(dim=1)).sum().item())


def time_batched(w, torch, calls: int = 100, nsub: int = 10, reps: int = 3):
    """Uneven swarm sizes: the persistent bucketed launch, autotuned, a
    rollout of ``calls`` calls of ``nsub`` substeps (observation after each
    call into its own slot) captured as one graph and replayed once per
    episode; plus the one-substep launch on the same swarms."""
    from paper_2306_09537_amd.quadswarm import QuadSwarm
    sim = QuadSwarm.from_workload(w)
    Q = w.n_quads
    acts = torch.from_numpy(w.action_sequence(calls)).cuda()
    goals = torch.from_numpy(w.goals).cuda()
    obs = torch.empty((calls, Q, w.obs_dim), device="cuda")
    s0 = torch.from_numpy(w.state0).cuda()
    choice = sim.autotune(acts[0], nsub, goals, obs[0])
    sim.set_graph_mode(True)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for c in range(calls):
            sim.step_observe(acts[c], nsub, goals, obs[c])
    times = []
    for r in range(reps + 1):
        # episode reset (untimed); every replay runs the same seeded episode
        sim.set_state(s0, 0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        if r:
            times.append(e0.elapsed_time(e1))
    nonfinite = sticky_nonfinite(sim, torch)
    sim.set_graph_mode(False)
    ms = float(np.median(times))
    value = Q * calls * nsub / (ms * 1e-3)
    # the one-substep launch (observation every substep) on the same swarms
    plain_ms, _ = time_calls(sim, w, acts, goals, obs[0], 1, 500, 20, torch, w.substeps)
    plain = Q / (plain_ms * 1e-3)
    sim.close()
    out = dict(workload=w.name, quads=Q, envs=w.n_envs, calls=calls, substeps_per_call=nsub,
               value=value, unit="quad-steps/s", ms_per_rollout=ms, autotune=choice,
               nonfinite_quads=nonfinite,
               form="persistent bucketed launch, 10 substeps per call, 100-call rollout "
                    "replayed as one captured graph",
               plain_value=plain, speedup_vs_plain=value / plain)
    # ALU roofline of one 10-substep call (counters of the autotuned launch)
    if (w.name, calls, nsub) == ("uneven_16384", 100, 10):
        rl = alu_roofline("bucket_kernel_uneven16384.md",
                          f"batched_b{choice['block']}_", ms / calls)
        if rl is not None:
            out["roofline"] = rl
    return out


def cpu_baseline(w, target_s: float):
    """The FP64 oracle on the host cores: step + observe per substep over a
    bounded number of substeps of the same workload."""
    from oracle import oracle as O
    orc = O.Oracle.from_workload(w)
    s0 = w.state0.astype(np.float64)
    s = s0
    g = w.goals.astype(np.float64)
    acts = [w.actions(i).astype(np.float64) for i in range(100)]
    t0 = time.perf_counter()
    n = 0
    while True:
        if n and n % 1000 == 0:
            s = s0  # episode reset, as on the GPU
        s, _, _ = orc.step(s, acts[n % 100], 1, n)
        orc.observe(s, g)
        n += 1
        if time.perf_counter() - t0 >= target_s:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=w.n_quads * n / dt, unit="quad-steps/s", cores=cores, kind="oracle",
                sample=f"{w.name}: {n} substeps x {w.n_quads} quads (step + K-NN observe per "
                       f"substep), FP64, {dt:.1f} s")


def cpu_table(seconds: float = 3.0) -> dict:
    """The FP64 oracle on the host cores for every configuration, each on a
    bounded sample (the first envs of the workload, a few substeps):
    quad-steps/s forward (step + K-NN observe per substep) and, for the
    differentiation workloads, forward + backward (the oracle's reverse mode
    re-runs its forward, so its whole time counts)."""
    from oracle import oracle as O
    from paper_2306_09537_amd import workloads as W

    def fwd(w, e1, max_sub):
        orc = O.Oracle.from_workload(w, 0, e1)
        q = int(w.env_offsets[e1])
        s = w.state0[:q].astype(np.float64)
        g = w.goals[:q].astype(np.float64)
        acts = [np.ascontiguousarray(w.actions(i)[:q], dtype=np.float64) for i in range(16)]
        t0 = time.perf_counter()
        n = 0
        while n < max_sub and (n == 0 or time.perf_counter() - t0 < seconds):
            s, _, _ = orc.step(s, acts[n % 16], 1, n)
            orc.observe(s, g)
            n += 1
        dt = time.perf_counter() - t0
        return dict(value=q * n / dt, sample=f"{e1} envs ({q} quads) x {n} substeps, {dt:.2f} s")

    def fwd_bwd(w, e1, T):
        orc = O.Oracle.from_workload(w, 0, e1)
        q = int(w.env_offsets[e1])
        rng = np.random.default_rng(0)
        acts = rng.uniform(0.05, 0.95, size=(T, q, 4))
        wt = rng.normal(size=(q, 27))
        gp = np.ones(q)
        t0 = time.perf_counter()
        orc.rollout_vjp(w.state0[:q].astype(np.float64), acts, 1, 0, wt, gp, 100.0)
        dt = time.perf_counter() - t0
        return dict(value=q * T / dt, sample=f"{e1} envs ({q} quads) x {T} substeps, {dt:.2f} s")

    rows = {
        "plain_64x1": fwd(W.plain(seed=0), 64, 20000),
        "swarm_4096x8": fwd(W.swarm8(seed=0), 4096, 1000),
        "uneven_16384": fwd(W.uneven(seed=0), 16384, 1000),
        "scale_1048576x1": fwd(W.scale1(seed=0), 1048576, 1000),
        "scale_32768x32": fwd(W.scale32(seed=0), 4096, 1000),
        "diff_1024x8 fwd+bwd": fwd_bwd(W.diff(seed=0), 1024, 200),
        "scale_32768x32 fwd+bwd": fwd_bwd(W.scale32(seed=0), 512, 100),
    }
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"cpu_table": rows, "unit": "quad-steps/s", "cores": cores, "kind": "oracle",
            "precision": "f64"}


def main():
    args = parse()
    if args.cpu_table:
        print(json.dumps(cpu_table()), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the swarm step has no cross-GPU exchange "
              "(environments are independent); run one process per GPU on disjoint "
              "environment ranges instead.", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4}))
        return

    from paper_2306_09537_amd import workloads as W
    from paper_2306_09537_amd.quadswarm import QuadSwarm

    torch.cuda.set_device(0)
    w = W.WORKLOADS[args.workload](seed=0)
    sim = QuadSwarm.from_workload(w)
    n_act = args.steps + args.warmup
    acts = torch.from_numpy(w.action_sequence(n_act)).cuda()  # a fresh action set per call
    goals = torch.from_numpy(w.goals).cuda()
    obs = torch.empty((w.n_quads, w.obs_dim), device="cuda")

    ms, wall_ms = time_calls(sim, w, acts, goals, obs, args.nsub, args.steps,
                             args.warmup, torch, w.substeps)
    kern_ms = ms
    Q = w.n_quads
    value = Q * args.nsub / (ms * 1e-3)
    bpq = algorithmic_bytes_per_quad(w.k_neighbors, args.nsub)
    launch_bytes = bpq * Q
    achieved = launch_bytes / (kern_ms * 1e-3) / 1e9

    extra = {}
    for ns in [int(x) for x in args.extra_nsub.split(",") if x.strip()]:
        if ns == args.nsub:
            continue
        sim2 = QuadSwarm.from_workload(w)
        m2, _ = time_calls(sim2, w, acts, goals, obs, ns, max(args.steps // ns, 20),
                           max(args.warmup // ns, 5), torch, w.substeps)
        sim2.close()
        extra[f"fused_nsub{ns}"] = dict(
            value=Q * ns / (m2 * 1e-3), ms_per_call=m2,
            speedup_vs_plain=(Q * ns / (m2 * 1e-3)) / value)
        rl = valu_roofline(args.workload, ns, m2)
        if rl is not None:
            extra[f"fused_nsub{ns}"]["roofline"] = rl

    traffic = launch_traffic(args.workload, args.nsub)
    line = {
        "metric": "quad-steps/s fwd at 1 MI355X (% of HBM roofline)",
        "value": value,
        "unit": "quad-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded: domain-randomised params, random initial states, U[0,1] actions)",
        "config": {"workload": w.name, "envs": w.n_envs, "quads": Q,
                   "k_neighbors": w.k_neighbors, "substeps_per_call": args.nsub,
                   "dt": w.consts["dt"], "entry": "qs_step_observe"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     # the counters' bytes over the same launch time: below the
                     # algorithmic rate where data stays in the 256 MB cache
                     "traffic_achieved": (traffic / (kern_ms * 1e-3) / 1e9
                                          if traffic else None),
                     "traffic_frac": (traffic / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      if traffic else None),
                     "kernel": "step_kernel (fused step + observe)",
                     "kernel_ms": kern_ms, "bytes_per_launch": launch_bytes,
                     "bytes_per_quad": bpq},
        "host_ms_per_step": wall_ms,
        "fused": extra,
    }
    if args.fwdbwd:
        wd = W.WORKLOADS[args.fwdbwd](seed=0)
        line["fwd_bwd"] = time_fwd_bwd(wd, torch, args.fwdbwd_horizon, 1, 20, 3)
    if args.batched:
        line["batched"] = time_batched(W.WORKLOADS[args.batched](seed=0), torch)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    sim.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
