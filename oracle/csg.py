"""Per-column Boolean operations on dexel grids, and the shell (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only callers allowed.  Nothing here is
shared with the GPU library.

A dexel shape is a set of closed z-intervals per column.  CSG on dexels works
column by column (Sec. 2, item (3): CSG carried out directly in dexel space),
and the shell of a shape is the Boolean difference of its dilation and its
erosion (Sec. 4, "3D Printing"; Fig. 1).

The operations are the regularised ones of solid modelling: the result is
the closure of the interior of the set operation, so a piece of zero length
(two intervals that only touch, or a difference that leaves a single point)
is dropped, and touching result pieces are one interval.  That is evaluated
here from its definition, without any interval sweep: the endpoints of both
columns cut the z-axis into elementary open segments; a segment is in the
result iff its midpoint is, by the set operation applied to membership in A
and in B; consecutive member segments form one closed interval.  Every
endpoint of the inputs is a float32 value, so the float64 midpoint of two
distinct endpoints lies strictly between them.
"""
from __future__ import annotations

import numpy as np

OPS = ("union", "intersect", "difference")


def _inside(iv: np.ndarray, m: float) -> bool:
    """m lies in the interior of one of the closed intervals iv[k] = (lo, hi)."""
    return bool(np.any((iv[:, 0] < m) & (m < iv[:, 1]))) if len(iv) else False


def column_op(a, b, op: str):
    """Regularised union / intersection / difference of two columns.

    a, b: arrays of shape (k, 2) (any order; overlapping allowed).  Returns a
    list of (lo, hi) with lo < hi, sorted, pairwise separated by a gap."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 2)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 2)
    pts = np.unique(np.concatenate([a.reshape(-1), b.reshape(-1)]))
    out = []
    for p, q in zip(pts[:-1], pts[1:]):
        m = 0.5 * (p + q)
        ia, ib = _inside(a, m), _inside(b, m)
        keep = {"union": ia or ib, "intersect": ia and ib, "difference": ia and not ib}[op]
        if not keep:
            continue
        if out and out[-1][1] == p:
            out[-1] = (out[-1][0], q)
        else:
            out.append((p, q))
    return out


def csg(ga, gb, op: str):
    """Column-by-column Boolean operation of two grids of the same size;
    returns (col_ptr int64[nx*ny+1], z float64[2n])."""
    if op not in OPS:
        raise ValueError(op)
    if (ga.nx, ga.ny) != (gb.nx, gb.ny):
        raise ValueError("grids differ in size")
    ncols = ga.nx * ga.ny
    col_ptr = np.zeros(ncols + 1, np.int64)
    z = []
    for c in range(ncols):
        ca = ga.z[2 * ga.col_ptr[c]: 2 * ga.col_ptr[c + 1]].reshape(-1, 2)
        cb = gb.z[2 * gb.col_ptr[c]: 2 * gb.col_ptr[c + 1]].reshape(-1, 2)
        res = column_op(ca, cb, op)
        col_ptr[c + 1] = col_ptr[c] + len(res)
        for lo, hi in res:
            z += [lo, hi]
    return col_ptr, np.asarray(z, dtype=np.float64)


def shell(grid, r: float, mode: str = "f64"):
    """S_shell = D_r(S) minus E_r(S) (Sec. 4, "3D Printing"), with D and E
    from the oracle's dilation and erosion in the given precision."""
    import oracle
    d = oracle.run(grid, r, "dilate", mode)
    e = oracle.run(grid, r, "erode", mode)
    return csg(d, e, "difference")
