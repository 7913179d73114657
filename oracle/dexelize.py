"""Dexelisation of analytic primitives (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only callers allowed.  Nothing here is
shared with the GPU library or with the input generators.

A dexel structure stores the intersections of a solid with parallel rays
cast from a uniform 2D grid (Sec. 1; Sec. 3.1, "Dexel Representation").
Readings: the rays are the z-parallel lines through the cell centres
(x + 0.5, y + 0.5) of an nx x ny grid; a ball (centre c, radius R) meets the
ray of a cell when the squared lateral distance rho2 = (x + 0.5 - cx)^2 +
(y + 0.5 - cy)^2 is below R^2, in the closed chord [cz - h, cz + h],
h = sqrt(R^2 - rho2); an axis-aligned box [a, b] meets the ray of a cell
whose integer index x satisfies ceil(ax - 0.5) <= x <= floor(bx - 0.5) (the
centre lies in [ax, bx]), and likewise in y, in the closed interval
[az, bz].  Every chord end is computed in float64 (products, sums and the
square root each rounded once, no fused operations), rounded once to
float32, and the float32 intervals of a column are merged where they
overlap or touch.  Footprints outside the grid are clipped; z is not.

Primitive records: (kind, a0, a1, a2, b0, b1, b2) with kind 0 = ball (a =
centre, b0 = radius) and kind 1 = box (a = low corner, b = high corner).

Rays along another axis (dexel structures in three orthogonal directions,
the "Limitations" paragraph of Sec. 4, and Sec. 5): for rays along axis k the grid's two axes
are (k + 1) mod 3 and (k + 2) mod 3, in that order, and the intervals lie
along k; so rays along x give a grid over (y, z), rays along y one over
(z, x).  The rules above then apply to the coordinates in that order.
"""
from __future__ import annotations

import math

import numpy as np

BALL, BOX = 0, 1


def column_intervals(x: int, y: int, prims):
    """Float32-rounded chords of every primitive on the ray of cell (x, y)."""
    px, py = x + 0.5, y + 0.5
    out = []
    for p in prims:
        kind = int(p[0])
        if kind == BALL:
            cx, cy, cz, R = float(p[1]), float(p[2]), float(p[3]), float(p[4])
            dx, dy = px - cx, py - cy
            rho2 = dx * dx + dy * dy
            if rho2 < R * R:
                h = math.sqrt(R * R - rho2)
                out.append((float(np.float32(cz - h)), float(np.float32(cz + h))))
        elif kind == BOX:
            ax, ay, az, bx, by, bz = (float(v) for v in p[1:7])
            if math.ceil(ax - 0.5) <= x <= math.floor(bx - 0.5) and \
                    math.ceil(ay - 0.5) <= y <= math.floor(by - 0.5):
                out.append((float(np.float32(az)), float(np.float32(bz))))
        else:
            raise ValueError(f"unknown primitive kind {kind}")
    return out


def merge(intervals):
    """Sort by start; an interval starting at or before the running end joins it."""
    res = []
    for lo, hi in sorted(intervals):
        if res and lo <= res[-1][1]:
            res[-1] = (res[-1][0], max(res[-1][1], hi))
        else:
            res.append((lo, hi))
    return res


AXES = {"x": 0, "y": 1, "z": 2}


def ray_frame(p, axis: str):
    """Record p with its coordinates taken as (grid axis 1, grid axis 2,
    along the ray); a ball's radius is not a coordinate and stays."""
    k = AXES[axis]
    order = ((k + 1) % 3, (k + 2) % 3, k)
    a = [p[1 + i] for i in order]
    if int(p[0]) == BOX:
        b = [p[4 + i] for i in order]
    else:
        b = list(p[4:7])
    return (p[0], *a, *b)


def dexelize(nx: int, ny: int, prims, axis: str = "z"):
    """CSR (col_ptr int64[nx*ny+1], z float64[2n]) of the union of the
    primitives, sampled by rays along `axis`."""
    prims = [ray_frame(tuple(p), axis) for p in np.asarray(prims, dtype=np.float64).reshape(-1, 7)]
    col_ptr = np.zeros(nx * ny + 1, np.int64)
    z = []
    for y in range(ny):
        for x in range(nx):
            iv = merge(column_intervals(x, y, prims))
            col_ptr[y * nx + x + 1] = col_ptr[y * nx + x] + len(iv)
            for lo, hi in iv:
                z += [lo, hi]
    return col_ptr, np.asarray(z, dtype=np.float64)
