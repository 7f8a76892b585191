"""Throughput benchmark of the batched quadrotor-swarm step on one MI355X.

Default workload: 4096 environments x 8 quadrotors (32,768 quads), full
physics (motor lag and noise, walls, floor, in-env collisions) and the K = 6
nearest-neighbour observation, dt = 5 ms.  One timed "step" is one call of
the whole hot path over the batch: ``qs_step_observe`` with ``--nsub``
substeps (default 1: every row of the path, including the observation, runs
once per substep), on inputs already resident in HBM.

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
STATE_B, PARAM_B, ACT_B, GOAL_B = 108, 24, 16, 12


def algorithmic_bytes_per_quad(k: int, nsub: int, with_obs: bool = True) -> int:
    """Bytes one call must move per quad: state in and out, parameters,
    action, and (with the observation) goal and obs row."""
    b = 2 * STATE_B + PARAM_B + ACT_B
    if with_obs:
        b += GOAL_B + 4 * (18 + 6 * k)
    return b


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="swarm8",
                    choices=["swarm8", "plain", "uneven", "diff", "scale32", "scale1"])
    ap.add_argument("--nsub", type=int, default=1, help="substeps per call")
    ap.add_argument("--extra-nsub", default="2,10",
                    help="also time these fused substep counts (comma list, '' for none)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def time_calls(sim, acts, goals, obs, nsub, steps, warmup, torch):
    """Returns (ms per call over the timed region, mean kernel ms from
    per-launch events)."""
    for i in range(warmup):
        sim.step_observe(acts[i % acts.shape[0]], nsub, goals, obs)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for i in range(steps):
        sim.step_observe(acts[(warmup + i) % acts.shape[0]], nsub, goals, obs)
    end.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    ms = start.elapsed_time(end)
    # per-launch duration: events bracketing each launch on the same stream
    n = min(steps, 200)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    for i in range(n):
        ev[i][0].record()
        sim.step_observe(acts[i % acts.shape[0]], nsub, goals, obs)
        ev[i][1].record()
    torch.cuda.synchronize()
    kern = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    sim.sync()
    return ms / steps, kern, wall / steps


def cpu_baseline(w, target_s: float):
    """The FP64 oracle on the host cores: step + observe per substep over a
    bounded number of substeps of the same workload."""
    from oracle import oracle as O
    orc = O.Oracle.from_workload(w)
    s = w.state0.astype(np.float64)
    g = w.goals.astype(np.float64)
    a = w.actions(0).astype(np.float64)
    t0 = time.perf_counter()
    n = 0
    while True:
        s, _, _ = orc.step(s, a, 1, n)
        orc.observe(s, g)
        n += 1
        if time.perf_counter() - t0 >= target_s:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=w.n_quads * n / dt, unit="quad-steps/s", cores=cores, kind="oracle",
                sample=f"{w.name}: {n} substeps x {w.n_quads} quads (step + K-NN observe per "
                       f"substep), FP64, {dt:.1f} s")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the swarm step has no cross-GPU exchange "
              "(environments are independent); run one process per GPU on disjoint "
              "environment ranges instead.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2306_09537_amd import workloads as W
    from paper_2306_09537_amd.quadswarm import QuadSwarm

    torch.cuda.set_device(0)
    w = W.WORKLOADS[args.workload](seed=0)
    sim = QuadSwarm.from_workload(w)
    n_act = min(args.steps + args.warmup, 256)
    acts = torch.from_numpy(w.action_sequence(n_act)).cuda()
    goals = torch.from_numpy(w.goals).cuda()
    obs = torch.empty((w.n_quads, w.obs_dim), device="cuda")

    ms, kern_ms, wall_ms = time_calls(sim, acts, goals, obs, args.nsub, args.steps,
                                      args.warmup, torch)
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
        m2, k2, _ = time_calls(sim2, acts, goals, obs, ns, max(args.steps // ns, 20),
                               args.warmup // 2, torch)
        sim2.close()
        extra[f"fused_nsub{ns}"] = dict(
            value=Q * ns / (m2 * 1e-3), ms_per_call=m2, kernel_ms=k2,
            speedup_vs_plain=(Q * ns / (m2 * 1e-3)) / value)

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "step_kernel (fused step + observe)",
                     "kernel_ms": kern_ms, "bytes_per_launch": launch_bytes,
                     "bytes_per_quad": bpq},
        "host_ms_per_step": wall_ms,
        "fused": extra,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    sim.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
