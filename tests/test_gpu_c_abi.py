"""A C99 program drives the library with no Python or PyTorch in the process
(device memory from the HIP runtime's C API): its step + observation of 4
colliding swarms of 8 quads, two substeps, must match the oracle.  The
program is built by the package build next to its source."""
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_09537_amd import workloads as W
from tests.c_abi import build_smoke

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def read_output(path):
    b = open(path, "rb").read()
    o = 0

    def take(dtype, n):
        nonlocal o
        a = np.frombuffer(b, dtype=dtype, count=n, offset=o)
        o += a.nbytes
        return a

    magic, Q, E, K, nsub, od = (int(v) for v in take(np.int32, 6))
    assert magic == 0x51534331
    flags = int(take(np.uint32, 1)[0])
    seed = int(take(np.uint64, 1)[0])
    t = int(take(np.uint64, 1)[0])
    cf = take(np.float32, 19).astype(np.float64)
    consts = dict(W.BASE_CONSTS)
    consts.update(dt=cf[0], gravity=cf[1], arm_length=cf[2], k_tau=cf[3], drag_coef=cf[4],
                  floor_mu=cf[5], motor_noise_decay=cf[6], motor_noise_std=cf[7],
                  room_min=tuple(cf[8:11]), room_max=tuple(cf[11:14]), wall_restitution=cf[14],
                  col_dist=cf[15], col_decay=cf[16], col_noise_v=cf[17], col_noise_w=cf[18])
    offs = take(np.int32, E + 1).copy()
    arr = {}
    for name, cols in (("params", 6), ("state0", 27), ("actions", 4), ("goals", 3),
                       ("state", 27), ("obs", od)):
        arr[name] = take(np.float32, Q * cols).reshape(Q, cols).astype(np.float64)
    assert o == len(b)
    return dict(Q=Q, K=K, nsub=nsub, flags=flags, seed=seed, t=t, consts=consts, offs=offs, **arr)


def test_c_program_matches_oracle(tmp_path):
    if not os.path.exists(build_smoke.EXE):
        pytest.fail(f"{build_smoke.EXE} is missing: run the package build first")
    out = tmp_path / "abi_smoke.bin"
    p = subprocess.run([build_smoke.EXE, str(out)], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    r = read_output(out)
    assert r["t"] == r["nsub"]
    orc = O.Oracle(r["offs"], r["consts"], r["params"], r["K"], r["flags"], r["seed"])
    ref, contacts, ev = orc.step(r["state0"], r["actions"], r["nsub"], 0)
    assert np.any(ev & O.EV_PAIR_RESPONSE)          # the swarms did collide
    fmax = 0.25 * r["params"][:, 0:1] * r["consts"]["gravity"] * r["params"][:, 4:5]
    floor = np.ones_like(ref)
    floor[:, W.SE:W.SE + 4] = fmax
    err = np.abs(r["state"] - ref) / np.maximum(np.abs(ref), floor)
    assert err.max() < 1e-5, err.max()
    # teacher-forced observation: the oracle observes the program's state
    ref_obs, _ = orc.observe(r["state"], r["goals"])
    oerr = np.abs(r["obs"] - ref_obs) / np.maximum(np.abs(ref_obs), 1.0)
    assert oerr.max() < 1e-6, oerr.max()
