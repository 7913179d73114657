"""Pins of the oracle's canonical form of per-column interval lists (CPU).

* hand-worked columns (overlap, touching ends, nesting, duplicates, points);
* brute force: at random points that are not endpoints, and at every
  endpoint, membership in the canonical list equals membership in some input
  interval; the result is sorted and pairwise separated;
* invariance under reordering the input, and idempotence;
* invalid intervals are rejected.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import canonical as oc


@pytest.mark.parametrize("pairs,want", [
    ([], []),
    ([(3, 4), (0, 1)], [(0, 1), (3, 4)]),
    ([(0, 2), (1, 3)], [(0, 3)]),
    ([(1, 3), (0, 2)], [(0, 3)]),
    ([(0, 1), (1, 2)], [(0, 2)]),                    # touching ends join
    ([(0, 10), (2, 3), (4, 5)], [(0, 10)]),           # nested
    ([(2, 3), (2, 3)], [(2, 3)]),                     # duplicates
    ([(5, 5), (1, 2)], [(1, 2), (5, 5)]),             # a point stays a point
    ([(2, 2), (1, 2)], [(1, 2)]),                     # a point on an end joins
    ([(4, 6), (0, 1), (1, 4)], [(0, 6)]),             # a chain in any order
    ([(-3, -1), (-1.5, 0.5), (7, 8)], [(-3, 0.5), (7, 8)]),
])
def test_worked_columns(pairs, want):
    assert oc.column(pairs) == [(float(a), float(b)) for a, b in want]


def _member(iv, z):
    return any(lo <= z <= hi for lo, hi in iv)


@pytest.mark.parametrize("seed", range(5))
def test_membership_brute_force(seed):
    rng = np.random.default_rng(seed)
    for _ in range(40):
        k = int(rng.integers(0, 25))
        lo = np.round(rng.uniform(0, 100, k), 1)
        hi = lo + np.round(rng.exponential(4.0, k), 1) * (rng.random(k) > 0.1)
        pairs = list(zip(lo, hi))
        res = oc.column(pairs)
        for (_, h0), (l1, _) in zip(res[:-1], res[1:]):
            assert h0 < l1
        for a, b in res:
            assert a <= b
        ends = {float(v) for p in pairs for v in p}
        zs = [z for z in rng.uniform(-5, 110, 300) if z not in ends] + sorted(ends)
        for z in zs:
            assert _member(res, z) == _member(pairs, z), (pairs, z)


@pytest.mark.parametrize("seed", range(3))
def test_order_invariance_and_idempotence(seed):
    rng = np.random.default_rng(50 + seed)
    nx, ny = 7, 5
    counts = rng.integers(0, 12, nx * ny)
    col_ptr = np.concatenate([[0], np.cumsum(counts)])
    lo = rng.uniform(0, 50, col_ptr[-1]).astype(np.float32).astype(np.float64)
    hi = lo + rng.uniform(0, 8, col_ptr[-1]).astype(np.float32).astype(np.float64)
    z = np.stack([lo, hi], 1).reshape(-1)
    cp, cz = oc.canonicalize(nx, ny, col_ptr, z)
    # shuffle every column's intervals
    pairs = z.reshape(-1, 2).copy()
    for c in range(nx * ny):
        a, b = col_ptr[c], col_ptr[c + 1]
        pairs[a:b] = pairs[a:b][rng.permutation(b - a)]
    cp2, cz2 = oc.canonicalize(nx, ny, col_ptr, pairs.reshape(-1))
    assert np.array_equal(cp, cp2) and np.array_equal(cz, cz2)
    cp3, cz3 = oc.canonicalize(nx, ny, cp, cz)
    assert np.array_equal(cp, cp3) and np.array_equal(cz, cz3)


@pytest.mark.parametrize("bad", [(2.0, 1.0), (float("nan"), 1.0), (0.0, float("inf"))])
def test_invalid_rejected(bad):
    with pytest.raises(ValueError):
        oc.column([(0.0, 1.0), bad])
