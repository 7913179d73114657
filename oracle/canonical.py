"""Canonical form of per-column interval lists (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only callers allowed.  Nothing here is
shared with the GPU library.

A dexel column is a set of closed z-intervals (Sec. 3.1, "Dexel
Representation").  Its canonical form, the input form of every offset call,
lists that set as sorted, pairwise separated closed intervals: the union of
the given intervals, with intervals that overlap or touch joined.  Given in
any order and overlapping freely, the intervals of a column are sorted by
(start, end) and swept once: an interval that starts at or before the
running end extends it, any other starts a new interval.  An interval with
start > end, or a non-finite end, makes the column invalid.
"""
from __future__ import annotations

import math

import numpy as np


def column(pairs):
    """Canonical list of one column's closed intervals (a list of (lo, hi))."""
    items = [(float(a), float(b)) for a, b in pairs]
    for a, b in items:
        if not (math.isfinite(a) and math.isfinite(b)) or a > b:
            raise ValueError(f"invalid interval ({a}, {b})")
    out = []
    for a, b in sorted(items):
        if out and a <= out[-1][1]:
            out[-1] = (out[-1][0], max(out[-1][1], b))
        else:
            out.append((a, b))
    return out


def canonicalize(nx: int, ny: int, col_ptr, z):
    """CSR (col_ptr int64[nx*ny+1], z float64[2n]) of the canonical form of a
    grid whose columns hold intervals in any order."""
    col_ptr = np.asarray(col_ptr, dtype=np.int64)
    z = np.asarray(z, dtype=np.float64).reshape(-1)
    ncols = nx * ny
    out_ptr = np.zeros(ncols + 1, np.int64)
    out = []
    for c in range(ncols):
        a, b = int(col_ptr[c]), int(col_ptr[c + 1])
        res = column(z[2 * a: 2 * b].reshape(-1, 2))
        out_ptr[c + 1] = out_ptr[c] + len(res)
        for lo, hi in res:
            out += [lo, hi]
    return out_ptr, np.asarray(out, dtype=np.float64)
