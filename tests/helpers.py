"""Small state-building helpers for tests (no simulator arithmetic)."""
import numpy as np

from paper_2306_09537_amd import workloads as W


def blank_state(q, z=5.0):
    s = np.zeros((q, W.STATE_DIM))
    s[:, 2] = z
    s[:, W.SR:W.SR + 9] = np.eye(3).reshape(9)
    return s


def rot_z(psi):
    c, s = np.cos(psi), np.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def nominal_params(q, **over):
    p = np.tile(np.array([W.NOMINAL[k] for k in
                          ("mass", "ixx", "iyy", "izz", "thrust_to_weight", "motor_tau")]), (q, 1))
    names = ("mass", "ixx", "iyy", "izz", "thrust_to_weight", "motor_tau")
    for k, v in over.items():
        p[:, names.index(k)] = v
    return p


def consts(**over):
    c = dict(W.BASE_CONSTS)
    c.update(over)
    return c
