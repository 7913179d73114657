"""GPU parity of the tri-dexel offset: a solid dexelised along x, y and z
(three orthogonal dexel structures: the "Limitations" paragraph of Sec. 4,
and Sec. 5), each structure offset by the same ball, through the C ABI.

* Each direction, bit-exact against the oracle: its dexelisation along that
  axis, then its offset in the float32 model; and within tolerance of FP64.
* A property that holds at any size: a set closed under the cyclic rotation
  of the axes looks the same along x, y and z, so the three grids, and their
  offsets, are bit-identical.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import dexelize as od
from tests.helpers import HostGrid, compare_columns

pytestmark = pytest.mark.gpu

GRIDS = {"x": lambda n: (n[1], n[2]), "y": lambda n: (n[2], n[0]), "z": lambda n: (n[0], n[1])}


def _prims(rng, ext, count, smax):
    out = []
    for _ in range(count):
        c = rng.uniform(-2, np.asarray(ext, dtype=np.float64) + 2)
        if rng.random() < 0.5:
            out.append((od.BALL, *c, rng.uniform(0.5, smax), 0.0, 0.0))
        else:
            out.append((od.BOX, *c, *(c + rng.uniform(0.0, 2 * smax, 3))))
    return out


@pytest.mark.parametrize("op,r", [("dilate", 3.5), ("erode", 2.0), ("close", 2.5)])
def test_each_direction_against_the_oracle(engine, oracle_lib, op, r):
    rng = np.random.default_rng(3)
    dims = (40, 33, 27)
    prims = _prims(rng, dims, 150, 5.0)
    print(f"[case] tridexel {op} r={r} dims={dims}", flush=True)
    tri = engine.tridexel(dims, np.asarray(prims))
    res = engine.tridexel_offset(tri, r, op)
    k = 2 if op in ("open", "close") else 1
    for axis in ("x", "y", "z"):
        nu, nv = GRIDS[axis](dims)
        assert (tri[axis].nx, tri[axis].ny) == (nu, nv)
        cp, z = od.dexelize(nu, nv, prims, axis=axis)
        src = HostGrid(nu, nv, cp, z)
        col, zz = tri[axis].to_host()
        assert np.array_equal(col, cp) and np.array_equal(zz.astype(np.float64), z), axis
        col, zz = res[axis].to_host()
        zz = zz.astype(np.float64)
        ref32 = oracle_lib.run(src, r, op, "f32model")
        assert np.array_equal(col, ref32.col_ptr), axis
        assert np.array_equal(zz, ref32.z), axis
        ref = oracle_lib.run(src, r, op, "f64")
        cmp = compare_columns(np.diff(ref.col_ptr), ref.z, np.diff(col), zz, r, k=k)
        assert cmp["failed"] == 0, (axis, cmp)


def test_rotation_closed_set_is_the_same_along_every_axis(engine):
    """256^3 cells; every primitive is added with its two cyclic rotations
    (x, y, z) -> (y, z, x) -> (z, x, y), so the union is invariant and the
    x-, y- and z-ray grids coincide, before and after a dilation."""
    rng = np.random.default_rng(8)
    n = 256
    base = _prims(rng, (n, n, n), 200, 24.0)
    prims = []
    for p in base:
        a, b = list(p[1:4]), list(p[4:7])
        for s in range(3):
            ra = a[s:] + a[:s]
            rb = (b[s:] + b[:s]) if p[0] == od.BOX else b
            prims.append((p[0], *ra, *rb))
    print("[case] tridexel rotation-closed set 256^3", flush=True)
    tri = engine.tridexel((n, n, n), np.asarray(prims))
    res = engine.tridexel_offset(tri, 6.0, "dilate")
    for d in (tri, res):
        cz, zz = d["z"].to_host()
        assert cz[-1] > 50000
        for axis in ("x", "y"):
            c, z = d[axis].to_host()
            assert np.array_equal(c, cz) and np.array_equal(z, zz), axis
