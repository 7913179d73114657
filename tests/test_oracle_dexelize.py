"""Pins of the oracle's dexelisation of analytic primitives (CPU).

* hand-derived columns of one box and one ball;
* brute force: at points of each ray farther than 1e-3 from every primitive's
  boundary, membership in the dexel union equals membership in a primitive,
  decided by the primitives' own inequalities (not by chords);
* the summed chord lengths of a ball approach its volume;
* agreement with the synthetic generator's separate, vectorised dexelisation
  of the same primitives.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import dexelize as od
from synth import gen


def _col(col_ptr, z, c):
    return [(float(z[2 * k]), float(z[2 * k + 1])) for k in range(col_ptr[c], col_ptr[c + 1])]


def test_one_box():
    # centres x + 0.5 in [1.2, 4.7] -> x = 1..4; y + 0.5 in [0.3, 2.9] -> y = 0..2
    cp, z = od.dexelize(6, 4, [(od.BOX, 1.2, 0.3, -1.0, 4.7, 2.9, 3.0)])
    for y in range(4):
        for x in range(6):
            want = [(-1.0, 3.0)] if (1 <= x <= 4 and y <= 2) else []
            assert _col(cp, z, y * 6 + x) == want, (x, y)


def test_one_ball_at_a_cell_centre():
    # centre (2.5, 2.5, 0), R = 1.5: the centre column, four neighbours at
    # distance 1, four diagonal cells at distance sqrt(2); distance 2 is out
    cp, z = od.dexelize(5, 5, [(od.BALL, 2.5, 2.5, 0.0, 1.5, 0.0, 0.0)])
    f = lambda v: float(np.float32(v))
    h1, h2 = f(math.sqrt(1.25)), f(0.5)
    for y in range(5):
        for x in range(5):
            d2 = (x - 2) ** 2 + (y - 2) ** 2
            want = {0: [(-1.5, 1.5)], 1: [(-h1, h1)], 2: [(-h2, h2)]}.get(d2, [])
            assert _col(cp, z, y * 5 + x) == want, (x, y)


def _inside(prim, x, y, zz):
    kind = int(prim[0])
    if kind == od.BALL:
        cx, cy, cz, R = prim[1:5]
        return (x - cx) ** 2 + (y - cy) ** 2 + (zz - cz) ** 2 < R * R
    ax, ay, az, bx, by, bz = prim[1:7]
    return ax <= x <= bx and ay <= y <= by and az <= zz <= bz


def _boundary_dist(prim, x, y, zz):
    kind = int(prim[0])
    if kind == od.BALL:
        cx, cy, cz, R = prim[1:5]
        return abs(math.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (zz - cz) ** 2) - R)
    ax, ay, az, bx, by, bz = prim[1:7]
    return min(abs(x - ax), abs(x - bx), abs(y - ay), abs(y - by), abs(zz - az), abs(zz - bz))


def _world(axis, u, v, t):
    """The world point at grid position (u, v) and ray coordinate t."""
    return {"z": (u, v, t), "x": (t, u, v), "y": (v, t, u)}[axis]


@pytest.mark.parametrize("axis", ["z", "x", "y"])
@pytest.mark.parametrize("seed", range(3))
def test_membership_brute_force(seed, axis):
    """Membership along each ray is decided by the primitives' inequalities
    at the world point, written per axis without the oracle's reordering."""
    rng = np.random.default_rng(seed)
    nu, nv = 12, 9
    prims = []
    for _ in range(10):
        if rng.random() < 0.5:
            prims.append((od.BALL, *rng.uniform(0, 12, 3), rng.uniform(1, 4), 0.0, 0.0))
        else:
            lo = rng.uniform(0, 12, 3)
            prims.append((od.BOX, *lo, *(lo + rng.uniform(1, 5, 3))))
    cp, z = od.dexelize(nu, nv, prims, axis=axis)
    hits = 0
    for v in range(nv):
        for u in range(nu):
            iv = _col(cp, z, v * nu + u)
            for t in rng.uniform(-5, 17, 60):
                p = _world(axis, u + 0.5, v + 0.5, t)
                if min(_boundary_dist(q, *p) for q in prims) < 1e-3:
                    continue
                truth = any(_inside(q, *p) for q in prims)
                hits += truth
                assert any(lo <= t <= hi for lo, hi in iv) == truth, (u, v, t)
    assert hits > 100


def test_box_along_each_axis():
    """One box [1.2, 4.7] x [0.3, 2.9] x [-1, 3]: rays along x see the y-z
    footprint and the x extent, rays along y the z-x footprint."""
    box = [(od.BOX, 1.2, 0.3, -1.0, 4.7, 2.9, 3.0)]
    cp, z = od.dexelize(4, 5, box, axis="x")      # grid (y, z): y = 0..2, z + 0.5 in [-1, 3] -> z = 0..2
    for v in range(5):
        for u in range(4):
            want = [(1.2, 4.7)] if (u <= 2 and v <= 2) else []
            assert _col(cp, z, v * 4 + u) == [tuple(float(np.float32(w)) for w in iv) for iv in want], (u, v)
    cp, z = od.dexelize(5, 6, box, axis="y")      # grid (z, x): z = 0..2, x = 1..4
    for v in range(6):
        for u in range(5):
            want = [(0.3, 2.9)] if (u <= 2 and 1 <= v <= 4) else []
            assert _col(cp, z, v * 5 + u) == [tuple(float(np.float32(w)) for w in iv) for iv in want], (u, v)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_rotated_set_matches_z(axis):
    """Rotating every primitive so that the ray axis takes z's place gives,
    bit for bit, the z-ray grid of the original set."""
    rng = np.random.default_rng(11)
    prims = []
    for _ in range(25):
        if rng.random() < 0.5:
            prims.append((od.BALL, *rng.uniform(0, 20, 3), rng.uniform(1, 5), 0.0, 0.0))
        else:
            lo = rng.uniform(0, 20, 3)
            prims.append((od.BOX, *lo, *(lo + rng.uniform(1, 6, 3))))
    # world (x, y, z) -> coordinates whose (grid 1, grid 2, ray) frame is (x, y, z)
    rot = {"x": lambda a: (a[2], a[0], a[1]), "y": lambda a: (a[1], a[2], a[0])}[axis]
    moved = []
    for p in prims:
        a = rot(p[1:4])
        b = rot(p[4:7]) if p[0] == od.BOX else p[4:7]
        moved.append((p[0], *a, *b))
    c0, z0 = od.dexelize(20, 20, prims)
    c1, z1 = od.dexelize(20, 20, moved, axis=axis)
    assert np.array_equal(c0, c1) and np.array_equal(z0, z1)


@pytest.mark.parametrize("axis", ["z", "x", "y"])
def test_ball_volume_each_axis(axis):
    R = 20.0
    cp, z = od.dexelize(64, 64, [(od.BALL, 32.1, 31.7, 30.4, R, 0.0, 0.0)], axis=axis)
    vol = float(np.sum(z[1::2] - z[0::2]))
    assert abs(vol / (4.0 / 3.0 * math.pi * R ** 3) - 1.0) < 0.01


def test_ball_volume():
    R = 20.0
    cp, z = od.dexelize(64, 64, [(od.BALL, 32.1, 31.7, 5.0, R, 0.0, 0.0)])
    vol = float(np.sum(z[1::2] - z[0::2]))
    assert abs(vol / (4.0 / 3.0 * math.pi * R ** 3) - 1.0) < 0.01


def test_agrees_with_generator():
    rec = gen.primitive_records(3, n=48, count=60, smin=2.0, smax=12.0)
    g = gen.primitives_grid(3, n=48, count=60, smin=2.0, smax=12.0)
    cp, z = od.dexelize(48, 48, rec)
    assert np.array_equal(cp, g.col_ptr)
    assert np.array_equal(z, np.asarray(g.z, dtype=np.float64).reshape(-1))
