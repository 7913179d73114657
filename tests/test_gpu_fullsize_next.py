"""GPU parity at benchmark size for dexelisation, the canonical form and the
tri-dexel structures, on sampled output columns that the oracle computes one
by one (a whole 2048^2 grid of 5400 primitives would take the pure-Python
oracle hours).  The calls are the ones bench.py times, on the same inputs.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import canonical as oc
from oracle import dexelize as od
from synth import gen

pytestmark = pytest.mark.gpu

N, COUNT = 2048, 5400
SOUP = dict(n=N, count=COUNT, smin=16.0, smax=256.0, height=float(N))


def _sample(rng, nx, ny, k):
    """k random columns plus the four corners and the middle of each border."""
    xs = list(rng.integers(0, nx, k)) + [0, nx - 1, 0, nx - 1, nx // 2, nx // 2, 0, nx - 1]
    ys = list(rng.integers(0, ny, k)) + [0, 0, ny - 1, ny - 1, 0, ny - 1, ny // 2, ny // 2]
    return list(zip((int(x) for x in xs), (int(y) for y in ys)))


def _column(col, z, c):
    return [(float(z[2 * k]), float(z[2 * k + 1])) for k in range(int(col[c]), int(col[c + 1]))]


@pytest.fixture(scope="module")
def soup(engine):
    rec = gen.primitive_records(7, **SOUP)
    print("[case] dexelize 2048^2 soup of 5400 primitives", flush=True)
    g = engine.dexelize(N, N, rec)
    col, z = g.to_host()
    return rec, col, z.astype(np.float64)


def test_dexelize_bench_soup_sampled(soup):
    rec, col, z = soup
    prims = [tuple(p) for p in rec]
    rng = np.random.default_rng(1)
    for x, y in _sample(rng, N, N, 300):
        want = od.merge(od.column_intervals(x, y, prims))
        assert _column(col, z, y * N + x) == want, (x, y)


def test_canonicalize_bench_grid(engine, soup):
    """The benchmark's input: every interval of the soup split at its float32
    midpoint and every column reversed.  The canonical form is the soup again
    (whole grid), and sampled columns equal the oracle's."""
    rec, cp, z = soup
    pairs = z.reshape(-1, 2).astype(np.float32)
    mid = (np.float32(0.5) * (pairs[:, 0] + pairs[:, 1])).astype(np.float32)
    halves = np.stack([np.stack([pairs[:, 0], mid], 1), np.stack([mid, pairs[:, 1]], 1)], 1).reshape(-1, 2)
    cp2 = 2 * cp
    col_of = np.repeat(np.arange(N * N), np.diff(cp2))
    j = np.arange(cp2[-1])
    messy = halves[cp2[col_of] + cp2[col_of + 1] - 1 - j]
    del halves, col_of, j
    print("[case] canonicalize 2048^2 split and reversed", flush=True)
    col, out = engine.canonicalize(N, N, cp2, messy.reshape(-1)).to_host()
    assert np.array_equal(col, cp)
    assert np.array_equal(out.astype(np.float64), z)
    rng = np.random.default_rng(2)
    for x, y in _sample(rng, N, N, 300):
        c = y * N + x
        want = oc.column(messy[cp2[c]:cp2[c + 1]].astype(np.float64))
        assert _column(col, out, c) == want, (x, y)


def test_tridexel_bench_soup_sampled(engine):
    """The c2 primitives in [0, 512]^3 dexelised along x, y and z, as the
    tri-dexel benchmark does; sampled columns of each direction against the
    oracle's dexelisation along that axis."""
    rec = gen.primitive_records(0)
    print("[case] tridexel 512^3 soup", flush=True)
    tri = engine.tridexel((512, 512, 512), rec)
    rng = np.random.default_rng(3)
    for axis in ("x", "y", "z"):
        prims = [od.ray_frame(tuple(p), axis) for p in rec]
        col, z = tri[axis].to_host()
        z = z.astype(np.float64)
        for u, v in _sample(rng, 512, 512, 150):
            want = od.merge(od.column_intervals(u, v, prims))
            assert _column(col, z, v * 512 + u) == want, (axis, u, v)
