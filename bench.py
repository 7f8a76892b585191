"""Throughput benchmark of the batched quadrotor-swarm step on one MI355X.

Headline: 32768 environments x 32 quadrotors (1,048,576 quads), full physics
(motor lag and noise, walls, floor, in-env collisions) and the K = 6
nearest-neighbour observation, dt = 5 ms, domain randomisation -- the
largest single-GPU configuration.  One timed "step" is one call of the whole
hot path over the batch: ``qs_step_observe`` with one substep (every row of
the path, including the observation, runs once per substep), on inputs
already resident in HBM.  value = quad-steps/s (quads x substeps / s).

The same JSON line carries the other forms and workloads:
  fused     the headline workload with 2 and 10 substeps per call;
  fwd_bwd   the headline workload's differentiable rollout (100 substeps,
            checkpoint every 20 calls, collision penalty) and its reverse pass;
  scale1    1,048,576 single-quad environments (K = 0), 1 and 10 substeps;
  swarm8    4096 x 8 (K = 6), 1 and 10 substeps;
  batched   16384 environments of uneven sizes 1..32, a 100-call rollout of
            10-substep calls replayed from a captured graph;
  diff      1024 x 8 differentiable rollout of 200 substeps;
  cpu_baseline  the FP64 oracle on the host cores, on a sample of the
            headline workload (median of 3, all cores and one core).

Rooflines: a one-substep launch moves ~340-484 B per quad for ~250-670
arithmetic operations, so it is bound by HBM (8 TB/s); its ``achieved`` is
algorithmic bytes per launch over the event-timed launch duration.  The
multi-substep forms re-use the state in registers and are bound by the
vector ALUs; their ``achieved`` is the algorithmic FP operations of the
method per second -- counted by the op-counting build of the FP64 oracle
(profiles/alg_flops.md) -- against the FP32 vector peak of 157.3 TFLOP/s.
Counter-measured HBM bytes and VALU instruction counts come from the
committed rocprofv3 summaries and are reported only while the kernel
sources still hash to the value they were taken at.
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
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector peak (256 CUs x 128 lanes x 2 x 2.4 GHz)
SIMD_GCYCLES_PER_S = 256 * 4 * 2.4   # VALU issue slots: 1024 SIMDs at 2.4 GHz
METRIC = "quad-steps/s fwd and fwd+bwd at 1 MI355X; % of HBM/VALU roofline"
KERNEL_SOURCES = tuple(f"paper_2306_09537_amd/csrc/{f}" for f in
                       ("qs_device.h", "qs_kernels.h", "qs_rollout.h", "qs_adjoint.h"))
STATE_B, PARAM_B, ACT_B, GOAL_B = 108, 24, 16, 12
ALG_FLOPS = "alg_flops.md"
# committed rocprofv3 summary per workload (kernel trace, HBM and VALU counters)
PROFILES = {"scale32": "step_kernel_scale32768x32.md",
            "scale1": "step_kernel_scale1048576x1.md",
            "swarm8": "step_kernel_swarm4096x8.md",
            "uneven": "bucket_kernel_uneven16384.md",
            "scale32_fwdbwd": "rollout_reverse_scale32768x32.md",
            "diff_fwdbwd": "rollout_reverse_diff1024x8.md"}
WORKLOAD_KEYS = {"plain_64x1": "plain", "swarm_4096x8": "swarm8", "uneven_16384": "uneven",
                 "diff_1024x8": "diff", "scale_32768x32": "scale32",
                 "scale_1048576x1": "scale1"}


def algorithmic_bytes_per_quad(k: int, nsub: int, with_obs: bool = True) -> int:
    """Bytes one call must move per quad: state in and out, parameters,
    action, and (with the observation) goal and obs row.  Independent of
    the number of substeps: the state stays in registers between them."""
    b = 2 * STATE_B + PARAM_B + ACT_B
    if with_obs:
        b += GOAL_B + 4 * (18 + 6 * k)
    return b


def backward_bytes(Q: int, horizon: int, nsub: int, ckpt_every: int) -> int:
    """Algorithmic bytes of one reverse pass: per quad-substep the tape
    written and read (2 x 124: state and motor-noise draws), the actions read
    twice (recompute and sweep) and the action gradient written; per segment
    its checkpoint and the parameters (read by the recompute); once the
    state adjoint in and out and the parameters and their gradient."""
    n_seg = (horizon + ckpt_every - 1) // ckpt_every
    return Q * horizon * nsub * (248 + 32 + 16) + Q * n_seg * (108 + 24) + Q * (216 + 80)


def kernel_source_hash() -> str:
    import hashlib
    m = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def profile_value(profile: str, key: str, need_hash: bool = True):
    """A "key: value" number from a committed summary under profiles/, or
    None (missing, or -- for counters -- taken on other kernel sources)."""
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    if need_hash and kernel_source_hash() not in text:
        return None
    for line in text.splitlines():
        line = line.strip()
        if line.startswith(key + ":"):
            v = line.split(":", 1)[1].strip()
            return float(v) if any(c in v for c in ".eE") else int(v)
    return None


def alg_flops(workload_name: str, what: str):
    """Algorithmic FP operations per unit (per quad-substep for step,
    rollout and fwdbwd; per quad for observe) from the op-counting oracle."""
    key = WORKLOAD_KEYS.get(workload_name)
    if key is None:
        return None
    return profile_value(ALG_FLOPS, f"{key}_{what}_flops", need_hash=False)


def call_flops(w, nsub: int, with_obs: bool = True):
    """Algorithmic FP operations of one call over the whole batch."""
    st = alg_flops(w.name, "step")
    ob = alg_flops(w.name, "observe") if with_obs else 0.0
    if st is None or ob is None:
        return None
    return w.n_quads * (nsub * st + ob)


def hbm_roofline(bytes_per_launch: int, ms: float, traffic=None, **extra) -> dict:
    ach = bytes_per_launch / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
           "traffic_achieved": traffic / (ms * 1e-3) / 1e9 if traffic else None,
           "traffic_frac": traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
           "bytes_per_launch": bytes_per_launch}
    out.update(extra)
    return out


def alu_roofline(flops, ms: float, profile=None, prefix: str = "", **extra):
    """Algorithmic FLOP/s against the FP32 vector peak; with the committed
    VALU counters of the same launch (if current), the kernel's instruction
    mix per algorithmic operation and its VALU issue utilisation as
    diagnostics."""
    if flops is None:
        return None
    s = ms * 1e-3
    tf = flops / s / 1e12
    out = {"bound": "alu", "achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": tf / FP32_PEAK_TFLOPS, "traffic": None, "alg_flops_per_call": flops}
    if profile:
        valu = profile_value(profile, prefix + "valu_insts")
        fp32 = profile_value(profile, prefix + "fp32_valu_insts")
        act = profile_value(profile, prefix + "active_inst_valu")
        traffic = profile_value(profile, prefix + "traffic_bytes")
        if traffic:
            out["traffic"] = traffic
        if valu:
            # wave64 instructions: 64 lane operations each
            out["valu_lane_ops_per_alg_flop"] = valu * 64 / flops
            out["fp32_lane_ops_per_alg_flop"] = (fp32 or 0) * 64 / flops
        if act:
            # SQ_ACTIVE_INST_VALU counts 4 cycles per instruction issued
            out["valu_issue_util"] = act * 4 / (s * SIMD_GCYCLES_PER_S * 1e9)
    out.update(extra)
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="scale32",
                    choices=["swarm8", "plain", "uneven", "diff", "scale32", "scale1"])
    ap.add_argument("--nsub", type=int, default=1, help="substeps per call")
    ap.add_argument("--extra-nsub", default="2,10",
                    help="also time these fused substep counts (comma list, '' for none)")
    ap.add_argument("--legs", default="fwd_bwd,scale1,swarm8,batched,diff",
                    help="extra legs (comma list of fwd_bwd, scale1, swarm8, batched, diff; "
                         "'' for none)")
    ap.add_argument("--fwdbwd-horizon", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=3.0,
                    help="length of each oracle CPU-baseline run")
    ap.add_argument("--no-cpu", action="store_true")
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


def step_leg(w, torch, nsubs, steps: int, warmup: int, plain_value=None):
    """One workload at several substep counts per call: value, ms per call,
    and the roofline of each form (HBM for one substep, ALU otherwise)."""
    from paper_2306_09537_amd.quadswarm import QuadSwarm
    key = WORKLOAD_KEYS.get(w.name)
    prof = PROFILES.get(key)
    Q = w.n_quads
    goals = torch.from_numpy(w.goals).cuda()
    obs = torch.empty((Q, w.obs_dim), device="cuda")
    out = {}
    for ns in nsubs:
        n_steps = max(steps // ns, 10) if ns > 1 else steps
        n_warm = max(warmup // ns, 3) if ns > 1 else warmup
        acts = torch.from_numpy(w.action_sequence(min(n_steps + n_warm, 64))).cuda()
        sim = QuadSwarm.from_workload(w)
        ms, wall = time_calls(sim, w, acts, goals, obs, ns, n_steps, n_warm, torch, w.substeps)
        sim.close()
        del acts
        v = Q * ns / (ms * 1e-3)
        r = {"value": v, "ms_per_call": ms, "host_ms_per_call": wall, "substeps_per_call": ns}
        flops = call_flops(w, ns)
        if ns == 1:
            plain_value = v
            bpq = algorithmic_bytes_per_quad(w.k_neighbors, ns)
            r["roofline"] = hbm_roofline(
                bpq * Q, ms, profile_value(prof, "plain_traffic_bytes") if prof else None,
                kernel="step_kernel (fused step + observe)", kernel_ms=ms, bytes_per_quad=bpq,
                alg_flops_per_call=flops,
                alg_tflops=flops / (ms * 1e-3) / 1e12 if flops else None)
        else:
            r["roofline"] = alu_roofline(flops, ms, prof, f"fused{ns}_")
            if plain_value:
                r["speedup_vs_plain"] = v / plain_value
        out[f"nsub{ns}"] = r
    return out


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
    del acts, gact, ckpt
    f, b = float(np.median(fwd)), float(np.median(bwd))
    steps = Q * horizon * nsub
    key = WORKLOAD_KEYS.get(w.name)
    prof = PROFILES.get(f"{key}_fwdbwd")
    fb = alg_flops(w.name, "fwdbwd")
    ro = alg_flops(w.name, "rollout")
    bb = backward_bytes(Q, horizon, nsub, ckpt_every)
    h_ok = prof is not None and profile_value(prof, "fwdbwd_horizon") == horizon
    return dict(
        workload=w.name, quads=Q, horizon_substeps=horizon * nsub, ckpt_every=ckpt_every,
        value=steps / ((f + b) * 1e-3), unit="quad-steps/s (fwd+bwd)",
        fwd_ms=f, bwd_ms=b, fwd_value=steps / (f * 1e-3),
        roofline=alu_roofline(fb * steps if fb else None, f + b,
                              prof if h_ok else None, "fwdbwd_",
                              note="algorithmic operations of the forward and its "
                                   "derivative over forward + backward time"),
        fwd_roofline=alu_roofline(ro * steps if ro else None, f, prof if h_ok else None,
                                  "rollout_"),
        bwd_roofline=hbm_roofline(
            bb, b, profile_value(prof, "backward_traffic_bytes") if h_ok else None,
            segment_substeps=ckpt_every * nsub))


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

    def replay_ms():
        """Capture the rollout as one graph and time its replays."""
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
        del graph
        return float(np.median(times)), nonfinite

    ms, nonfinite = replay_ms()
    # the same launch without the per-slot choices (every slot on the
    # one-partner body): what the autotuner's global search alone gives
    chunked = [r["slot"] for r in choice["slots"] if r["chunked"]]
    global_ms = ms
    if chunked:
        sim.set_partner_chunks([])
        global_ms, _ = replay_ms()
        sim.set_partner_chunks(chunked)
    value = Q * calls * nsub / (ms * 1e-3)
    # the one-substep launch (observation every substep) on the same swarms
    plain_ms, _ = time_calls(sim, w, acts, goals, obs[0], 1, 500, 20, torch, w.substeps)
    plain = Q / (plain_ms * 1e-3)
    sim.close()
    key = WORKLOAD_KEYS.get(w.name)
    return dict(workload=w.name, quads=Q, envs=w.n_envs, calls=calls, substeps_per_call=nsub,
                value=value, unit="quad-steps/s", ms_per_rollout=ms, autotune=choice,
                nonfinite_quads=nonfinite,
                form="persistent bucketed launch, 10 substeps per call, 100-call rollout "
                     "replayed as one captured graph",
                plain_value=plain, speedup_vs_plain=value / plain,
                global_choice_value=Q * calls * nsub / (global_ms * 1e-3),
                plain_roofline=hbm_roofline(algorithmic_bytes_per_quad(w.k_neighbors, 1) * Q,
                                            plain_ms),
                roofline=alu_roofline(call_flops(w, nsub), ms / calls, PROFILES.get(key),
                                      "fused10_"))


def _omp():
    """The OpenMP runtime the oracle links (thread count control)."""
    import ctypes
    from oracle import oracle as O
    O.lib()  # loads libgomp with the oracle
    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds: float, n_envs: int = 4096, runs: int = 3):
    """The FP64 oracle on the host cores: step + K-NN observe per substep
    on the first ``n_envs`` environments of the workload, each run bounded
    to ``seconds``; median of ``runs`` runs with every host core the
    process may use and with one core."""
    from oracle import oracle as O
    e1 = min(n_envs, w.n_envs)
    orc = O.Oracle.from_workload(w, 0, e1)
    q = int(w.env_offsets[e1])
    s0 = w.state0[:q].astype(np.float64)
    g = w.goals[:q].astype(np.float64)
    acts = [np.ascontiguousarray(w.actions(i)[:q], dtype=np.float64) for i in range(10)]

    def one_run():
        s = s0
        n = 0
        t0 = time.perf_counter()
        while n == 0 or time.perf_counter() - t0 < seconds:
            if n and n % w.substeps == 0:
                s = s0  # episode reset, as on the GPU
            s, _, _ = orc.step(s, acts[n % 10], 1, n)
            orc.observe(s, g)
            n += 1
        dt = time.perf_counter() - t0
        return q * n / dt, n, dt

    omp = _omp()
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    all_threads = omp.omp_get_max_threads() if omp else avail
    res = {}
    for label, nthr in (("all", all_threads), ("one", 1)):
        if omp:
            omp.omp_set_num_threads(int(nthr))
        rr = [one_run() for _ in range(runs)]
        res[label] = (float(np.median([r[0] for r in rr])), [r[0] for r in rr],
                      int(np.median([r[1] for r in rr])))
    if omp:
        omp.omp_set_num_threads(int(all_threads))
    v, vals, n = res["all"]
    v1, vals1, n1 = res["one"]
    return dict(value=v, unit="quad-steps/s", cores=int(all_threads), kind="oracle",
                sample=f"{w.name}: first {e1} envs ({q} quads), step + K-NN observe per substep, "
                       f"FP64, {runs} runs of {seconds:.0f} s each (median; ~{n} substeps per run "
                       f"on all cores, ~{n1} on one)",
                runs=vals, per_core=v / max(1, all_threads),
                one_core={"value": v1, "runs": vals1, "cores": 1},
                cpu_model=cpu_model(), host_cpus_available=avail,
                omp_proc_bind=os.environ.get("OMP_PROC_BIND", ""))


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
    omp = _omp()
    cores = omp.omp_get_max_threads() if omp else (os.cpu_count() or 1)
    return {"cpu_table": rows, "unit": "quad-steps/s", "cores": cores, "kind": "oracle",
            "precision": "f64", "cpu_model": cpu_model()}


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

    torch.cuda.set_device(0)
    w = W.WORKLOADS[args.workload](seed=0)
    extra = [int(x) for x in args.extra_nsub.split(",") if x.strip() and int(x) != args.nsub]
    head = step_leg(w, torch, [args.nsub], args.steps, args.warmup)[f"nsub{args.nsub}"]
    fused = step_leg(w, torch, extra, args.steps, args.warmup, plain_value=head["value"]) \
        if extra else {}
    Q = w.n_quads
    ms = head["ms_per_call"]
    roof = head["roofline"]
    if args.nsub != 1:  # a multi-substep headline is priced on the ALUs
        roof = alu_roofline(call_flops(w, args.nsub), ms, PROFILES.get(WORKLOAD_KEYS[w.name]),
                            f"fused{args.nsub}_")
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "quad-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded: domain-randomised params, random initial states, "
                "U[0,1] actions)",
        "config": {"workload": w.name, "envs": w.n_envs, "quads": Q,
                   "k_neighbors": w.k_neighbors, "substeps_per_call": args.nsub,
                   "dt": w.consts["dt"], "entry": "qs_step_observe"},
        "roofline": roof,
        "host_ms_per_step": head["host_ms_per_call"],
        "fused": fused,
    }
    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    if "fwd_bwd" in legs:
        line["fwd_bwd"] = time_fwd_bwd(w, torch, args.fwdbwd_horizon, 1, 20, 3)
        torch.cuda.empty_cache()
    if "scale1" in legs and w.name != "scale_1048576x1":
        line["scale1"] = dict(workload="scale_1048576x1",
                              **step_leg(W.scale1(seed=0), torch, [1, 10], args.steps,
                                         args.warmup))
        torch.cuda.empty_cache()
    if "swarm8" in legs and w.name != "swarm_4096x8":
        line["swarm8"] = dict(workload="swarm_4096x8",
                              **step_leg(W.swarm8(seed=0), torch, [1, 2, 10],
                                         max(args.steps, 200), args.warmup))
    if "batched" in legs:
        line["batched"] = time_batched(W.uneven(seed=0), torch)
    if "diff" in legs:
        line["diff"] = time_fwd_bwd(W.diff(seed=0), torch, 200, 1, 20, 3)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
