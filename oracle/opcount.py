"""Algorithmic floating-point work of the method per unit, from the
op-counting build of the oracle (``opcount.cpp``); writes
``profiles/alg_flops.md``.

MEASUREMENT INFRASTRUCTURE ONLY: it runs the oracle (nothing of the GPU
library) on samples of each workload and stores, per workload,

- ``<w>_step_flops``: FP operations per quad-substep of a step (motor,
  rigid body, walls, floor and the in-env pair pass), averaged over the
  first ten substeps of the workload's episode, one substep per call;
- ``<w>_observe_flops``: per quad of one observation (K nearest);
- ``<w>_rollout_flops`` and ``<w>_fwdbwd_flops``: per quad-substep of the
  differentiable rollout with the smoothed collision penalty, and of its
  reverse pass including the forward it needs (the oracle's reverse mode
  runs its forward once and differentiates it), for the workloads that have
  a fwd+bwd leg.

Every add, subtract, multiply, divide, square root and transcendental
counts as one operation (see ``opcount.cpp`` for what is left out).  The
samples are the first environments of each workload with its own seeded
initial state and actions.

    python -m oracle.opcount            # writes profiles/alg_flops.md
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "profiles", "alg_flops.md")
SUBSTEPS = 10
BETA = 100.0


def _counted(fn):
    from oracle import oracle as O
    O.opcount_reset()
    out = fn()
    return O.opcount_get(), out


def unit_counts(w, n_envs: int, fwdbwd: bool) -> dict:
    """Per-unit counts on the first n_envs environments of workload w."""
    from oracle import oracle as O
    orc = O.Oracle.from_workload(w, 0, n_envs)
    q = int(w.env_offsets[n_envs])
    s0 = w.state0[:q].astype(np.float64)
    g = w.goals[:q].astype(np.float64)
    acts = [w.actions(c)[:q].astype(np.float64) for c in range(SUBSTEPS)]

    def steps():
        s = s0
        for c in range(SUBSTEPS):
            s, _, _ = orc.step(s, acts[c], 1, c)
        return s
    st, s_end = _counted(steps)
    ob, _ = _counted(lambda: orc.observe(s_end, g))
    row = {"quads": q, "step": st["total"] / (SUBSTEPS * q), "observe": ob["total"] / q,
           "step_trans": st["trans"] / (SUBSTEPS * q), "step_sqrt": st["sqrt"] / (SUBSTEPS * q),
           "step_div": st["div"] / (SUBSTEPS * q)}
    if fwdbwd:
        a = np.stack(acts)
        rng = np.random.default_rng(0)
        wt = rng.normal(size=(q, 27))
        wt[:, 26] = 0.0
        gp = np.ones(q)
        ro, _ = _counted(lambda: orc.rollout(s0, a, 1, 0, beta=BETA))
        fb, _ = _counted(lambda: orc.rollout_vjp(s0, a, 1, 0, wt, gp, BETA))
        row["rollout"] = ro["total"] / (SUBSTEPS * q)
        row["fwdbwd"] = fb["total"] / (SUBSTEPS * q)
    return row


def main() -> None:
    from oracle import oracle as O
    os.environ["QS_ORACLE_LIB"] = O.build_opcount()
    sys.path.insert(0, ROOT)
    from paper_2306_09537_amd import workloads as W
    cases = [  # (key, workload, sample envs, fwd+bwd leg)
        ("plain", W.plain(seed=0), 64, False),
        ("swarm8", W.swarm8(seed=0), 512, False),
        ("uneven", W.uneven(seed=0), 1024, False),
        ("diff", W.diff(seed=0), 256, True),
        ("scale32", W.scale32(seed=0), 64, True),
        ("scale1", W.scale1(seed=0), 16384, False),
    ]
    lines = ["# Algorithmic FP operations per unit of work (op-counting oracle)", "",
             "Written by `python -m oracle.opcount` (the oracle's source compiled with a "
             "counting double, `oracle/opcount.cpp`): every add, subtract, multiply, divide, "
             "square root and transcendental of the plain FP64 definition counts one; "
             "comparisons, selects, the threshold-margin diagnostics, the per-quad constants "
             "(f_max, alpha_lag, ...) and the integer work of the noise generator do not.  "
             "Samples: the first environments of each workload, ten substeps of one-substep "
             "calls from its initial state.", "",
             "| Workload | sample quads | step / quad-substep | of which sqrt, div, transc. | "
             "observe / quad | rollout / quad-substep | fwd+bwd / quad-substep |",
             "|---|---|---|---|---|---|---|"]
    keys = []
    for key, w, ne, fb in cases:
        r = unit_counts(w, ne, fb)
        ro = f"{r['rollout']:.1f}" if fb else "—"
        fw = f"{r['fwdbwd']:.1f}" if fb else "—"
        lines.append(f"| {w.name} | {r['quads']} | {r['step']:.1f} | {r['step_sqrt']:.1f}, "
                     f"{r['step_div']:.1f}, {r['step_trans']:.1f} | {r['observe']:.1f} | "
                     f"{ro} | {fw} |")
        keys.append(f"{key}_step_flops: {r['step']:.3f}")
        keys.append(f"{key}_observe_flops: {r['observe']:.3f}")
        if fb:
            keys.append(f"{key}_rollout_flops: {r['rollout']:.3f}")
            keys.append(f"{key}_fwdbwd_flops: {r['fwdbwd']:.3f}")
    lines += ["", "Values read by `bench.py` (per quad-substep, or per quad for observe):", ""]
    lines += [f"    {k}" for k in keys]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
