"""Host check of the rounding argument behind the expanded partner screen
of swarms of 16 and 32 (the in-swarm pass, §III-B.1): for a quad with every
coordinate within 10 m, e = |b|^2 + (|a|^2 - thr_x) - 2 a.b evaluated in
float32 as the kernel evaluates it (three-term FMA chains, one add) is
negative for every partner in contact, thr_x being d_col^2 widened by three
times the bound 7 u ((|a| + |b|)^2 + d_col^2).  float32 FMAs are emulated
as float64 operations rounded once to float32 (the float32 product is exact
in float64; the float64 sum can round once more, which only loosens the
check by far less than the widening)."""
import numpy as np

U = 2.0 ** -24
BOX = 10.0


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def fma32(a, b, c):
    return f32(a * b + c)


def thr_x(dcol):
    reach = 2.0 * 1.7320508 * BOX + dcol + 1e-3
    err = 1.01 * 7.0 * 5.9604645e-8 * (reach * reach + dcol * dcol)
    return f32(f32(dcol * dcol) + 3.0 * err), err


def screen_e(a, b, dcol):
    t, _ = thr_x(dcol)
    nb = fma32(b[:, 2], b[:, 2], fma32(b[:, 1], b[:, 1], f32(b[:, 0] * b[:, 0])))
    na = fma32(a[:, 2], a[:, 2], fma32(a[:, 1], a[:, 1], fma32(a[:, 0], a[:, 0], -t)))
    s = f32(nb + na)
    return fma32(-2.0 * a[:, 2], b[:, 2], fma32(-2.0 * a[:, 1], b[:, 1], fma32(-2.0 * a[:, 0], b[:, 0], s)))


def contact_pairs(rng, m, dcol, lo, hi):
    a = f32(rng.uniform(lo, hi, size=(m, 3)))
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = dcol * (1.0 - rng.uniform(0.0, 1e-4, size=(m, 1)))  # just inside d_col
    b = f32(a + r * u)
    d2 = ((a - b) ** 2).sum(axis=1)
    keep = d2 < dcol * dcol
    return a[keep], b[keep]


def test_screen_keeps_contacts_at_the_box_corners():
    rng = np.random.default_rng(0)
    for dcol in (0.1, 0.05, 0.3):
        for lo, hi in ((-10.0, -9.5), (9.5, 10.0), (-10.0, 10.0)):
            a, b = contact_pairs(rng, 200_000, dcol, lo, hi)
            a = a[np.abs(a).max(axis=1) <= BOX]
            b = b[: len(a)]
            assert len(a) > 100_000
            assert (screen_e(a, b, dcol) < 0).all(), (dcol, lo, hi)


def test_rounding_stays_within_the_bound():
    rng = np.random.default_rng(1)
    dcol = 0.1
    t, err = thr_x(dcol)
    a = f32(rng.uniform(-BOX, BOX, size=(400_000, 3)))
    b = f32(a + rng.normal(scale=0.2, size=a.shape))
    exact = ((a - b) ** 2).sum(axis=1) - t
    bound = 7 * U * ((np.linalg.norm(a, axis=1) + np.linalg.norm(b, axis=1)) ** 2 + t)
    got = np.abs(screen_e(a, b, dcol) - exact)
    assert (got <= bound).all()
    # for pairs in contact the bound stays below err, and the widening is
    # three times err
    touching = ((a - b) ** 2).sum(axis=1) < dcol * dcol
    assert touching.sum() > 1000
    assert bound[touching].max() <= err and t - dcol * dcol >= 2.9 * err


def test_widening_is_small():
    # the screen keeps the exact test's work rare: about 7 mm at d_col = 0.1 m
    t, _ = thr_x(0.1)
    assert 0.1 < np.sqrt(t) < 0.108
