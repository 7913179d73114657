"""Pins of the FP64 oracle against what the paper and the mathematics fix.

The oracle computes dilation as the brute-force union of capsule chords
(Sec. 4 "Baseline Comparison"; Sec. 3.1 "Dilation" equation) and erosion as
complement-dilate-complement (Sec. 3.1 "Erosion").  These tests check it
against things that do not go through chords:

* hand-derived closed forms in tests/golden/closed_forms.json (Pythagorean
  radii, exact square roots);
* a point-sampled distance test: a sample is in the dilation iff some shape
  point is within r (squared lateral distance plus squared z distance to an
  interval), in the erosion iff no complement point of an in-grid column is
  within r -- a different formula from the oracle's chord construction;
* closed forms for boxes, slabs and dexelised balls, including the sphere
  sandwich  dexel(ball(R0+r-sqrt2)) <= D_r(dexel(ball R0)) <= dexel(ball(R0+r));
* invariants that hold exactly: extensivity, monotonicity in r,
  D(S u T) = D(S) u D(T), the symmetries of the square, r = 0 identity.

Non-square grids are used throughout so that an x/y transposition fails.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from tests.helpers import (HostGrid, grid_from_columns, intervals_membership, near_endpoint,
                           random_grid, sampled_membership)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _oracle_cols(oracle, g, r, op, mode="f64"):
    cnt, z = oracle.offset_columns(g, r, op, mode)
    z = z.reshape(-1, 2)
    off = np.concatenate([[0], np.cumsum(cnt)])
    return [z[off[c]:off[c + 1]] for c in range(g.nx * g.ny)]


# ---------------------------------------------------------------------------
# golden closed forms
# ---------------------------------------------------------------------------

def _golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"][:40])
def test_golden_closed_forms(oracle_lib, case):
    nx, ny = case["nx"], case["ny"]
    if "point" in case:
        px, py, pz = case["point"]
        cols = [[] for _ in range(nx * ny)]
        cols[py * nx + px] = [(pz, pz)]
    else:
        cols = [[tuple(iv) for iv in col] for col in case["columns"]]
    g = grid_from_columns(nx, ny, cols)
    out = _oracle_cols(oracle_lib, g, case["r"], case["op"])
    if "expect" in case:
        for c, exp in enumerate(case["expect"]):
            got = out[c]
            assert len(got) == len(exp), (c, got, exp)
            if exp:
                np.testing.assert_allclose(got, np.array(exp), rtol=0, atol=1e-12)
    else:
        for (x, y), exp in case["probe"]:
            got = out[y * nx + x]
            assert len(got) == len(exp), ((x, y), got, exp)
            if exp:
                np.testing.assert_allclose(got, np.array(exp), rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# point-sampled distance test (independent formula)
# ---------------------------------------------------------------------------

SAMPLED = [  # (nx, ny, height, radius)
    (7, 5, 24.0, 1.0), (9, 6, 32.0, 2.0), (6, 11, 32.0, 2.5), (10, 7, 32.0, 3.0),
    (8, 9, 28.0, 1.7320508), (12, 5, 32.0, 4.2), (5, 5, 16.0, 0.5), (11, 8, 32.0, 0.0),
]


@pytest.mark.parametrize("op", ["dilate", "erode"])
@pytest.mark.parametrize("nx,ny,height,r", SAMPLED)
def test_point_sampled(oracle_lib, nx, ny, height, r, op):
    rng = np.random.default_rng(1000 + nx * 31 + ny * 7 + int(r * 100))
    g = random_grid(rng, nx, ny, height, max_per_col=3, p_empty=0.25)
    r32 = float(np.float32(r))
    out = _oracle_cols(oracle_lib, g, r32, op)
    zs = np.linspace(-r32 - 2.0, height + r32 + 2.0, 1601) + 1.0 / 4096.0
    checked = 0
    for c in range(nx * ny):
        ref = sampled_membership(g, r32, op, c, zs)
        got = intervals_membership(out[c], zs)
        keep = ~near_endpoint(out[c], zs)
        bad = np.flatnonzero((ref != got) & keep)
        assert bad.size == 0, (c, zs[bad[:5]], out[c], g.column(c))
        checked += int(keep.sum())
    assert checked > nx * ny * 1000


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("r", [1.0, 2.0, 3.0, 2.6, 4.5])
def test_box_dilation_closed_form(oracle_lib, r):
    r = float(np.float32(r))  # the oracle receives the radius as float32
    nx, ny = 17, 13
    x0, x1, y0, y1, z0, z1 = 5, 9, 4, 7, 3.25, 11.5
    cols = [[(z0, z1)] if (x0 <= c % nx <= x1 and y0 <= c // nx <= y1) else []
            for c in range(nx * ny)]
    g = grid_from_columns(nx, ny, cols)
    out = _oracle_cols(oracle_lib, g, r, "dilate")
    for c in range(nx * ny):
        x, y = c % nx, c // nx
        d2 = max(0, x0 - x, x - x1) ** 2 + max(0, y0 - y, y - y1) ** 2
        if d2 <= r * r:
            h = math.sqrt(r * r - d2)
            np.testing.assert_allclose(out[c], [[z0 - h, z1 + h]], rtol=0, atol=1e-12)
        else:
            assert len(out[c]) == 0, (x, y, out[c])


@pytest.mark.parametrize("r", [1.0, 2.0, 2.6])
def test_box_erosion_closed_form(oracle_lib, r):
    r = float(np.float32(r))
    nx, ny = 19, 16
    x0, x1, y0, y1, z0, z1 = 4, 13, 4, 11, 2.0, 14.0
    cols = [[(z0, z1)] if (x0 <= c % nx <= x1 and y0 <= c // nx <= y1) else []
            for c in range(nx * ny)]
    g = grid_from_columns(nx, ny, cols)
    out = _oracle_cols(oracle_lib, g, r, "erode")
    R = int(math.floor(r))
    for c in range(nx * ny):
        x, y = c % nx, c // nx
        if x0 + R <= x <= x1 - R and y0 + R <= y <= y1 - R:
            np.testing.assert_allclose(out[c], [[z0 + r, z1 - r]], rtol=0, atol=1e-12)
        else:
            assert len(out[c]) == 0, (x, y, out[c])


@pytest.mark.parametrize("op,r,expect", [("dilate", 2.0, (1.0, 10.0)), ("erode", 2.0, (5.0, 6.0)),
                                         ("close", 2.0, (3.0, 8.0)), ("open", 2.0, (3.0, 8.0)),
                                         ("erode", 2.5, (5.5, 5.5)), ("open", 2.5, (0.0, 0.0))])
def test_slab(oracle_lib, op, r, expect):
    nx, ny = 6, 4
    g = grid_from_columns(nx, ny, [[(3.0, 8.0)]] * (nx * ny))
    res = oracle_lib.run(g, r, op)
    for c in range(nx * ny):
        col = res.column(c)
        lo, hi = expect
        if hi > lo:
            np.testing.assert_allclose(col, [[lo, hi]], rtol=0, atol=1e-12)
        else:
            assert len(col) == 0


def _ball_grid(n, cx, cy, cz, R0):
    cols = []
    for c in range(n * n):
        x, y = c % n + 0.5, c // n + 0.5
        rho2 = (x - cx) ** 2 + (y - cy) ** 2
        cols.append([(cz - math.sqrt(R0 * R0 - rho2), cz + math.sqrt(R0 * R0 - rho2))]
                    if rho2 <= R0 * R0 else [])
    return grid_from_columns(n, n, cols)


@pytest.mark.parametrize("R0,r", [(6.3, 2.0), (5.1, 3.7), (8.0, 1.0), (4.4, 4.4)])
def test_sphere_sandwich(oracle_lib, R0, r):
    """dexel(ball(R0 + r - sqrt2)) <= D_r(dexel(ball R0)) <= dexel(ball(R0 + r))."""
    n = int(2 * (R0 + r)) + 6
    cx = cy = n / 2.0 + 0.13
    cz = 20.0
    g = _ball_grid(n, cx, cy, cz, R0)
    out = _oracle_cols(oracle_lib, g, r, "dilate")
    inner = _ball_grid(n, cx, cy, cz, R0 + r - math.sqrt(2.0))
    outer = _ball_grid(n, cx, cy, cz, R0 + r)
    for c in range(n * n):
        got = out[c]
        for lo, hi in inner.column(c):
            assert any(a - 1e-9 <= lo and hi <= b + 1e-9 for a, b in got), (c, got, (lo, hi))
        for a, b in got:
            assert any(lo - 1e-9 <= a and b <= hi + 1e-9 for lo, hi in outer.column(c)), (c, got)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def _subset(A, B, eps=1e-12):
    """Every interval of A inside some interval of B (per column)."""
    for a_col, b_col in zip(A, B):
        for lo, hi in a_col:
            if hi - lo <= 0:
                continue
            if not any(a - eps <= lo and hi <= b + eps for a, b in b_col):
                return False
    return True


def _union_grid(g1, g2):
    cols = []
    for c in range(g1.nx * g1.ny):
        iv = sorted([tuple(v) for v in g1.column(c)] + [tuple(v) for v in g2.column(c)])
        m = []
        for lo, hi in iv:
            if m and lo <= m[-1][1]:
                m[-1] = (m[-1][0], max(hi, m[-1][1]))
            else:
                m.append((lo, hi))
        cols.append(m)
    return grid_from_columns(g1.nx, g1.ny, cols)


def _transform(g, kind):
    nx, ny = g.nx, g.ny
    if kind == "transpose":
        cols = [g.column(x * nx + y).tolist() for y in range(nx) for x in range(ny)]
        return grid_from_columns(ny, nx, cols)
    if kind == "flipx":
        cols = [g.column(y * nx + (nx - 1 - x)).tolist() for y in range(ny) for x in range(nx)]
        return grid_from_columns(nx, ny, cols)
    if kind == "flipy":
        cols = [g.column((ny - 1 - y) * nx + x).tolist() for y in range(ny) for x in range(nx)]
        return grid_from_columns(nx, ny, cols)
    raise KeyError(kind)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_invariants(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    g = random_grid(rng, 11, 7, 40.0, max_per_col=3)
    h = random_grid(rng, 11, 7, 40.0, max_per_col=2)
    for r in (1.0, 2.5, 3.0):
        D = _oracle_cols(oracle_lib, g, r, "dilate")
        E = _oracle_cols(oracle_lib, g, r, "erode")
        S = g.columns()
        assert _subset(S, D)                        # extensive
        assert _subset(E, S)                        # anti-extensive
        C = oracle_lib.run(g, r, "close")
        O = oracle_lib.run(g, r, "open")
        assert _subset(S, [C.column(c) for c in range(g.nx * g.ny)])
        assert _subset([O.column(c) for c in range(g.nx * g.ny)], S)
        D2 = _oracle_cols(oracle_lib, g, r + 0.75, "dilate")
        E2 = _oracle_cols(oracle_lib, g, r + 0.75, "erode")
        assert _subset(D, D2) and _subset(E2, E)  # monotone in r
        # D(S u T) = D(S) u D(T), exactly
        U = _oracle_cols(oracle_lib, _union_grid(g, h), r, "dilate")
        DT = _oracle_cols(oracle_lib, h, r, "dilate")
        DU = _union_grid(grid_from_columns(g.nx, g.ny, [d.tolist() for d in D]),
                         grid_from_columns(g.nx, g.ny, [d.tolist() for d in DT]))
        for c in range(g.nx * g.ny):
            np.testing.assert_array_equal(U[c], DU.column(c))
        # D_r(D_s(S)) inside D_{r+s}(S)
        DD = oracle_lib.run(oracle_lib.run(g, r, "dilate"), 1.5, "dilate")
        Drs = _oracle_cols(oracle_lib, g, r + 1.5, "dilate")
        assert _subset([DD.column(c) for c in range(g.nx * g.ny)], Drs, eps=1e-9)


@pytest.mark.parametrize("kind", ["transpose", "flipx", "flipy"])
@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_symmetry(oracle_lib, kind, op):
    rng = np.random.default_rng(7)
    g = random_grid(rng, 9, 6, 30.0, max_per_col=3)
    for r in (1.5, 3.0):
        a = _transform(grid_from_columns(g.nx, g.ny, [c.tolist() for c in _oracle_cols(oracle_lib, g, r, op)]), kind)
        t = _transform(g, kind)
        b = _oracle_cols(oracle_lib, t, r, op)
        for c in range(t.nx * t.ny):
            np.testing.assert_array_equal(a.column(c), b[c])


def test_radius_zero_identity(oracle_lib):
    rng = np.random.default_rng(3)
    g = random_grid(rng, 8, 5, 20.0)
    D = _oracle_cols(oracle_lib, g, 0.0, "dilate")
    E = _oracle_cols(oracle_lib, g, 0.0, "erode")
    for c in range(g.nx * g.ny):
        np.testing.assert_array_equal(D[c], g.column(c))
        # erosion by 0 keeps every positive-length interval
        keep = [iv for iv in g.column(c) if iv[1] > iv[0]]
        np.testing.assert_array_equal(E[c], np.array(keep).reshape(-1, 2))


def test_f32_model_within_tolerance(oracle_lib):
    """The float32 model differs from the f64 result only by rounding."""
    from tests.helpers import compare_columns
    rng = np.random.default_rng(11)
    g = random_grid(rng, 12, 9, 200.0, max_per_col=4)
    for r in (2.0, 3.3):
        for op in ("dilate", "erode"):
            c64, z64 = oracle_lib.offset_columns(g, r, op, "f64")
            c32, z32 = oracle_lib.offset_columns(g, r, op, "f32model")
            res = compare_columns(c64, z64, c32, z32, r)
            assert res["failed"] == 0, res


def test_region_chain_matches_full(oracle_lib):
    rng = np.random.default_rng(5)
    g = random_grid(rng, 14, 10, 30.0, max_per_col=3)
    for op in ("close", "open"):
        full = oracle_lib.run(g, 2.0, op)
        cols = np.array([0, 13, 27, 70, 139], dtype=np.int64)
        cnt, z = oracle_lib.region_chain(g, 2.0, op, cols)
        zz = z.reshape(-1, 2)
        off = np.concatenate([[0], np.cumsum(cnt)])
        for k, c in enumerate(cols):
            np.testing.assert_array_equal(zz[off[k]:off[k + 1]], full.column(c))
