"""Helpers shared by the GPU parity tests (comparison logic only)."""
import numpy as np

from paper_2306_09537_amd import workloads as W

TOL = 1e-5          # per-step relative error bound (state blocks with floors)
MARGIN = 1e-5       # threshold decisions this close may legitimately flip
CONTACT_TIE = 1e-6  # contact pairs this close to d_col may differ


def fmax_of(params):
    p = np.asarray(params, dtype=np.float64)
    return 0.25 * p[:, 0] * 9.81 * p[:, 4]


def rel_err(gpu, ref, fmax):
    """Per element |g - o| / max(|o|, floor): floors 1 m, 1 m/s, 1 (R, u),
    1 rad/s, f_max (motor noise), 1 (floor flag)."""
    floor = np.ones_like(ref)
    floor[:, W.SE:W.SE + 4] = fmax[:, None]
    return np.abs(np.asarray(gpu, np.float64) - ref) / np.maximum(np.abs(ref), floor)


def pair_dist(pos, offs, q, j_local):
    e_start = offs[np.searchsorted(offs, q, side="right") - 1]
    return np.linalg.norm(pos[q] - pos[e_start + j_local])


def check_contacts(c_gpu, c_ref, pos_gpu, pos_ref, offs, dcol):
    """Contact masks equal except for pairs within CONTACT_TIE of d_col."""
    c_gpu = np.asarray(c_gpu).astype(np.uint64)
    c_ref = np.asarray(c_ref).astype(np.uint64)
    diff = np.nonzero(c_gpu != c_ref)[0]
    ties = 0
    for q in diff:
        x = int(c_gpu[q] ^ c_ref[q])
        j = 0
        while x:
            if x & 1:
                dg = pair_dist(pos_gpu, offs, q, j)
                do = pair_dist(pos_ref, offs, q, j)
                assert min(abs(dg - dcol), abs(do - dcol)) < CONTACT_TIE, (q, j, dg, do)
                ties += 1
            x >>= 1
            j += 1
    return ties


def check_obs(obs_gpu, obs_ref, state, offs, K, tol=2e-6):
    """Observation rows equal to tol; a neighbour-slot mismatch is accepted
    only where distances tie within 1e-6 m and the GPU's slots are a valid
    nearest-K list of the same environment."""
    g = np.asarray(obs_gpu, np.float64)
    o = np.asarray(obs_ref, np.float64)
    assert g.shape == o.shape
    err = np.abs(g - o) / np.maximum(np.abs(o), 1.0)
    assert err[:, :18].max() <= tol, err[:, :18].max()
    if K == 0:
        return 0
    bad = np.nonzero(err[:, 18:].max(axis=1) > tol)[0]
    pos = state[:, 0:3].astype(np.float64)
    vel = state[:, W.SV:W.SV + 3].astype(np.float64)
    for q in bad:
        e = np.searchsorted(offs, q, side="right") - 1
        q0, q1 = offs[e], offs[e + 1]
        others = [j for j in range(q0, q1) if j != q]
        d = np.array([np.linalg.norm(pos[j] - pos[q]) for j in others])
        order = np.lexsort((np.arange(len(others)), d))
        kk = min(K, len(others))
        kth = d[order[kk - 1]]
        used = set()
        for k in range(kk):
            rel = g[q, 18 + 6 * k: 21 + 6 * k]
            match = [j for j in others if np.allclose(pos[j] - pos[q], rel, atol=tol, rtol=0)]
            assert len(match) >= 1, (q, k)
            j = match[0]
            assert j not in used
            used.add(j)
            assert np.allclose(g[q, 21 + 6 * k: 24 + 6 * k], vel[j] - vel[q], atol=tol)
            assert np.linalg.norm(pos[j] - pos[q]) <= kth + 1e-6
        # the tie really exists at the boundary
        dd = np.sort(d)
        assert np.any(np.abs(np.diff(dd[:kk + 1])) < 1e-6) if len(dd) > kk else True
        assert np.all(g[q, 18 + 6 * kk:] == 0.0)
    return len(bad)
