"""Pins of the oracle's per-column CSG and shell (CPU).

* hand-worked columns (overlap, touching ends, containment, identical inputs);
* brute force: at random points that are not endpoints, membership in the
  result equals the Boolean operation of the memberships in the inputs;
* identities of regularised set operations: (A - B) + (A * B) = A,
  commutativity of union and intersection, (A + B) - B = A - B;
* the shell: shell + E = D, shell * E = empty, shell - D = empty
  (E inside S inside D for r >= 0).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import csg
from tests.helpers import grid_from_columns, random_grid


def cols(res):
    return [tuple(map(float, iv)) for iv in res]


@pytest.mark.parametrize("a,b,op,want", [
    ([(0, 2), (3, 5)], [(1, 4)], "union", [(0, 5)]),
    ([(0, 2), (3, 5)], [(1, 4)], "intersect", [(1, 2), (3, 4)]),
    ([(0, 2), (3, 5)], [(1, 4)], "difference", [(0, 1), (4, 5)]),
    ([(1, 4)], [(0, 2), (3, 5)], "difference", [(2, 3)]),
    ([(0, 1)], [(1, 2)], "union", [(0, 2)]),            # touching ends merge
    ([(0, 1)], [(1, 2)], "intersect", []),              # a single point is dropped
    ([(0, 1)], [(1, 2)], "difference", [(0, 1)]),
    ([(0, 10)], [(2, 3), (5, 6)], "difference", [(0, 2), (3, 5), (6, 10)]),
    ([(2, 3), (5, 6)], [(0, 10)], "difference", []),
    ([(0, 1), (2, 3)], [(0, 1), (2, 3)], "difference", []),
    ([(0, 1), (2, 3)], [(0, 1), (2, 3)], "intersect", [(0, 1), (2, 3)]),
    ([(0, 1), (2, 3)], [(0, 1), (2, 3)], "union", [(0, 1), (2, 3)]),
    ([], [(0, 1)], "union", [(0, 1)]),
    ([], [(0, 1)], "difference", []),
    ([(0, 1)], [], "difference", [(0, 1)]),
    ([(-3, -1), (4, 9)], [(-2, 5)], "union", [(-3, 9)]),
    ([(-3, -1), (4, 9)], [(-2, 5)], "difference", [(-3, -2), (5, 9)]),
])
def test_worked_columns(a, b, op, want):
    assert cols(csg.column_op(a, b, op)) == want


def _canonical(res):
    for lo, hi in res:
        assert lo < hi
    for (_, h0), (l1, _) in zip(res[:-1], res[1:]):
        assert h0 < l1


def _member(iv, z):
    return any(lo <= z <= hi for lo, hi in iv)


@pytest.mark.parametrize("seed", range(6))
def test_membership_brute_force(seed):
    rng = np.random.default_rng(seed)
    g = random_grid(rng, 6, 5, 100.0, max_per_col=6, p_empty=0.2)
    h = random_grid(rng, 6, 5, 100.0, max_per_col=6, p_empty=0.2)
    ends = set(g.z.tolist()) | set(h.z.tolist())
    zs = [z for z in rng.uniform(-5, 105, 400) if z not in ends]
    for op, f in (("union", lambda p, q: p or q), ("intersect", lambda p, q: p and q),
                  ("difference", lambda p, q: p and not q)):
        for c in range(g.nx * g.ny):
            a, b = g.column(c), h.column(c)
            res = csg.column_op(a, b, op)
            _canonical(res)
            for z in zs:
                assert _member(res, z) == f(_member(a, z), _member(b, z)), (op, c, z)


@pytest.mark.parametrize("seed", range(4))
def test_identities(seed):
    rng = np.random.default_rng(100 + seed)
    g = random_grid(rng, 5, 4, 50.0, max_per_col=5, p_empty=0.2)
    h = random_grid(rng, 5, 4, 50.0, max_per_col=5, p_empty=0.2)
    for c in range(g.nx * g.ny):
        a, b = g.column(c), h.column(c)
        diff = csg.column_op(a, b, "difference")
        inter = csg.column_op(a, b, "intersect")
        back = csg.column_op(np.array(diff).reshape(-1, 2), np.array(inter).reshape(-1, 2), "union")
        assert cols(back) == cols(a)
        assert cols(csg.column_op(a, b, "union")) == cols(csg.column_op(b, a, "union"))
        assert cols(inter) == cols(csg.column_op(b, a, "intersect"))
        u = np.array(csg.column_op(a, b, "union")).reshape(-1, 2)
        assert cols(csg.column_op(u, b, "difference")) == cols(diff)


def _grid(col_ptr, z, like):
    return oracle.Grid(like.nx, like.ny, col_ptr, z)


@pytest.mark.parametrize("r", [1.0, 2.5])
def test_shell_identities(oracle_lib, r):
    rng = np.random.default_rng(7)
    g = random_grid(rng, 9, 8, 40.0, max_per_col=4, p_empty=0.25)
    d = oracle.run(g, r, "dilate", "f64")
    e = oracle.run(g, r, "erode", "f64")
    sh = _grid(*csg.shell(g, r, "f64"), g)
    for c in range(g.nx * g.ny):
        s, ec, dc = sh.column(c), e.column(c), d.column(c)
        assert cols(csg.column_op(s, ec, "union")) == cols(dc)
        assert csg.column_op(s, ec, "intersect") == []
        assert csg.column_op(s, dc, "difference") == []


def test_shell_of_a_ball_column():
    """One column, one interval [0, 10], r = 2: dilation [-2, 12] (the column
    itself, no neighbours), erosion [2, 8]; the shell is [-2, 2] and [8, 12]."""
    g = grid_from_columns(1, 1, [[(0.0, 10.0)]])
    col_ptr, z = csg.shell(g, 2.0, "f64")
    assert list(col_ptr) == [0, 2]
    assert list(z) == [-2.0, 2.0, 8.0, 12.0]
