"""Block-wise comparison of a float32 gradient with the FP64 oracle's.

Every gradient is split into blocks that are checked on their own scale, so
that a small block (the thrust-to-weight column carries ~1e-5 of the
parameter gradient's norm on a dense swarm) cannot hide behind a large one:

- initial state: x, v, R, omega, u_f, eps (the resting flag has none);
- actions: one block per rotor;
- parameters: mass, ixx, iyy, izz, thrust-to-weight, tau_m.

Each block gets two checks against bounds derived from the oracle itself:
the oracle's gradient is recomputed from an initial state perturbed by
2^-23 relative noise (one float32 rounding), and the change this causes,
times 10, is the bound (with a floor):

- norm-wise: ||g - g_ref||_2 / ||g_ref||_2 <= max(1e-4, 10 ||g_pert - g_ref|| / ||g_ref||);
- element-wise, on the block's own scale: max|g - g_ref| / max|g_ref|
  <= max(2e-4, 10 max|g_pert - g_ref| / max|g_ref|).

A block whose reference is zero to double precision (norm below 1e-12 of
its family's: all state blocks, all rotors or all parameter columns) is
analytically zero -- e.g. the mass gradient of quads resting on the floor,
whose accelerations do not depend on the mass because the thrust scales
with it (f_max = m g t2w / 4) -- and the float32 path then holds only
rounding noise: its norm must stay below 1e-5 of the family's norm.  Every
other block, however small its share of the family (the thrust-to-weight
column carries ~1e-5 of the parameter gradient's norm), is checked on its
own scale as above.
"""
from __future__ import annotations

import numpy as np

STATE_BLOCKS = (("x", slice(0, 3)), ("v", slice(3, 6)), ("R", slice(6, 15)),
                ("omega", slice(15, 18)), ("u_f", slice(18, 22)), ("eps", slice(22, 26)))
PARAM_NAMES = ("mass", "ixx", "iyy", "izz", "t2w", "tau_m")
NORM_FLOOR = 1e-4
ELEM_FLOOR = 2e-4


def blocks(g_state, g_act, g_par):
    """(name, array) of every block of one gradient triple."""
    out = [("state." + n, np.asarray(g_state)[:, sl]) for n, sl in STATE_BLOCKS]
    ga = np.asarray(g_act)
    out += [(f"action.rotor{i}", ga[..., i]) for i in range(4)]
    gp = np.asarray(g_par)
    out += [("param." + n, gp[:, i]) for i, n in enumerate(PARAM_NAMES)]
    return out


def _norm(a):
    return float(np.linalg.norm(np.asarray(a, np.float64).ravel()))


def _amax(a):
    a = np.asarray(a, np.float64)
    return float(np.abs(a).max()) if a.size else 0.0


ZERO_REL = 1e-12    # reference block / family norm below this: analytically zero
NOISE_REL = 1e-5    # float32 noise allowed on such a block, relative to the family


def compare(got, ref, pert):
    """Rows (name, norm err, norm bound, elem err, elem bound, ok) for the
    gradient triples got (float32 path), ref (oracle) and pert (oracle from
    the perturbed initial state).  For an analytically zero block the norm
    columns hold ||g|| / family norm and its bound."""
    rows = []
    fam = {}
    for name, r in blocks(*ref):
        k = name.split(".")[0]
        fam[k] = fam.get(k, 0.0) + _norm(r) ** 2
    for (name, g), (_, r), (_, p) in zip(blocks(*got), blocks(*ref), blocks(*pert)):
        g = np.asarray(g, np.float64)
        r = np.asarray(r, np.float64)
        p = np.asarray(p, np.float64)
        nr, mr = _norm(r), _amax(r)
        nf = np.sqrt(fam[name.split(".")[0]])
        if nr <= ZERO_REL * nf:
            e = _norm(g) / nf if nf > 0 else _norm(g)
            b = NOISE_REL if nf > 0 else 0.0
            rows.append((name, e, b, e, b, bool(np.isfinite(e) and e <= b)))
            continue
        en = _norm(g - r) / nr
        bn = max(NORM_FLOOR, 10.0 * _norm(p - r) / nr)
        ee = _amax(g - r) / mr
        be = max(ELEM_FLOOR, 10.0 * _amax(p - r) / mr)
        rows.append((name, en, bn, ee, be, bool(np.isfinite(en) and en <= bn and ee <= be)))
    return rows


def failures(rows):
    return [r for r in rows if not r[5]]


def report(rows, title=""):
    lines = [f"{title}: block  norm-err / bound  elem-err / bound"]
    for name, en, bn, ee, be, ok in rows:
        lines.append(f"  {name:16s} {en:9.2e} / {bn:9.2e}  {ee:9.2e} / {be:9.2e}"
                     f"{'' if ok else '  FAIL'}")
    return "\n".join(lines)


def zeroed(got, block):
    """A copy of the gradient triple with one block set to zero (for the
    checks that a wrong column is caught)."""
    gs, ga, gp = (np.array(a, np.float64, copy=True) for a in got)
    kind, name = block.split(".")
    if kind == "state":
        gs[:, dict(STATE_BLOCKS)[name]] = 0.0
    elif kind == "action":
        ga[..., int(name[-1])] = 0.0
    else:
        gp[:, PARAM_NAMES.index(name)] = 0.0
    return gs, ga, gp
