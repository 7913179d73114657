"""GPU parity of dexel_canonicalize through the C ABI.

Endpoints are copied, never computed, so the bar is bit-exact against the
oracle (oracle/canonical.py): on grids it finishes in seconds, with columns
that take the LDS path and columns long enough for the sorting path; and, at
any size, on the property that a canonical grid is its own canonical form.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import canonical as oc
from synth import gen

pytestmark = pytest.mark.gpu


def _dx():
    import paper_1804_08968_amd as dx
    return dx


def _messy(rng, ncols, max_per_col, long_cols=()):
    """Columns of float32 intervals in random order: overlapping, nested,
    touching, duplicated and zero-length ones; some columns much longer."""
    counts = rng.integers(0, max_per_col + 1, ncols)
    for c in long_cols:
        counts[c] = 400 + 37 * (c % 5)
    col_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = int(col_ptr[-1])
    lo = np.round(rng.uniform(0, 300, n), 1).astype(np.float32)
    ln = np.round(rng.exponential(3.0, n), 1).astype(np.float32) * (rng.random(n) > 0.1)
    hi = (lo + ln).astype(np.float32)
    pairs = np.stack([lo, hi], 1)
    # touching and duplicated neighbours
    k = rng.random(n) < 0.1
    pairs[1:][k[1:], 0] = pairs[:-1][k[1:], 1]
    pairs[1:][k[1:], 1] = np.maximum(pairs[1:][k[1:], 0], pairs[1:][k[1:], 1])
    d = np.flatnonzero(rng.random(n) < 0.05)
    pairs[d[d > 0]] = pairs[d[d > 0] - 1]
    return col_ptr, pairs.reshape(-1)


def _check(engine, nx, ny, col_ptr, z):
    g = engine.canonicalize(nx, ny, col_ptr, z)
    col, out = g.to_host()
    rc, rz = oc.canonicalize(nx, ny, col_ptr, z.astype(np.float64))
    assert np.array_equal(col, rc)
    assert np.array_equal(out.astype(np.float64), rz)


@pytest.mark.parametrize("seed", range(3))
def test_random_columns(engine, seed):
    """Several 64-column blocks with a ragged tail; a few columns of 400+
    intervals take the sorting path, short columns whose running union
    passes 32 intervals too."""
    rng = np.random.default_rng(seed)
    nx, ny = 37, 11
    col_ptr, z = _messy(rng, nx * ny, 60, long_cols=(0, 5, 200, nx * ny - 1))
    print(f"[case] canonicalize random seed {seed}", flush=True)
    _check(engine, nx, ny, col_ptr, z)


def test_empty_and_one_column(engine):
    print("[case] canonicalize empty", flush=True)
    _check(engine, 4, 3, np.zeros(13, np.int64), np.zeros(0, np.float32))
    col_ptr = np.array([0, 5], np.int64)
    z = np.array([3, 4, 0, 1, 1, 2, 9, 9, 2, 2.5], np.float32)
    _check(engine, 1, 1, col_ptr, z)


def test_canonical_grid_is_unchanged(engine):
    """The 512^2 soup (canonical by construction) is its own canonical form;
    with every column's intervals reversed and split in two overlapping
    halves, its canonical form is the soup again."""
    g = gen.primitives_grid(0)
    print("[case] canonicalize soup 512^2", flush=True)
    out = engine.canonicalize(g.nx, g.ny, g.col_ptr, np.asarray(g.z, np.float32))
    col, z = out.to_host()
    assert np.array_equal(col, g.col_ptr)
    assert np.array_equal(z, np.asarray(g.z, np.float32).reshape(-1))
    pairs = np.asarray(g.z, np.float32).reshape(-1, 2)
    mid = (0.5 * (pairs[:, 0] + pairs[:, 1])).astype(np.float32)
    halves = np.stack([np.stack([pairs[:, 0], mid], 1), np.stack([mid, pairs[:, 1]], 1)], 1)
    cp = np.asarray(g.col_ptr)
    parts = []
    for c in range(g.nx * g.ny):
        a, b = cp[c], cp[c + 1]
        parts.append(halves[a:b].reshape(-1, 2)[::-1])
    z2 = np.concatenate(parts).reshape(-1)
    col, z = engine.canonicalize(g.nx, g.ny, 2 * cp, z2).to_host()
    assert np.array_equal(col, g.col_ptr)
    assert np.array_equal(z, np.asarray(g.z, np.float32).reshape(-1))


def test_errors_reported(engine):
    dx = _dx()
    print("[case] canonicalize errors", flush=True)
    col_ptr = np.array([0, 1, 2], np.int64)
    for bad in ([0, 1, 5, 4], [0, 1, np.nan, 4], [0, np.inf, 1, 2]):
        with pytest.raises(dx.DexelError) as e:
            engine.canonicalize(2, 1, col_ptr, np.array(bad, np.float32))
        assert e.value.status == dx.DEXEL_ERR_INVALID
    # a bad interval deep in a long column (after the LDS list ran out)
    z = np.stack([np.arange(100, dtype=np.float32) * 3, np.arange(100, dtype=np.float32) * 3 + 1], 1)
    z[90] = (5.0, 4.0)
    with pytest.raises(dx.DexelError) as e:
        engine.canonicalize(1, 1, np.array([0, 100], np.int64), z.reshape(-1))
    assert e.value.status == dx.DEXEL_ERR_INVALID
    # column pointers out of order, or not ending at nseg
    for cp in ([0, 2, 1], [0, 1, 1], [1, 1, 2]):
        with pytest.raises(dx.DexelError) as e:
            engine.canonicalize(2, 1, np.array(cp, np.int64), np.array([0, 1, 2, 3], np.float32))
        assert e.value.status == dx.DEXEL_ERR_INVALID
    # capacity: the output has room for fewer intervals than the result
    cp_d = torch.tensor([0, 1, 2], dtype=torch.int64, device="cuda")   # held: the view keeps raw pointers
    z_d = torch.tensor([0, 1, 2, 3], dtype=torch.float32, device="cuda")
    v = dx.make_view(2, 1, cp_d, z_d, 2)
    ws = torch.empty(dx.dexel_canonicalize_workspace_size(engine.ctx, v), dtype=torch.uint8, device="cuda")
    o = (torch.empty(3, dtype=torch.int64, device="cuda"), torch.empty(2, dtype=torch.float32, device="cuda"),
         torch.zeros(1, dtype=torch.int64, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"))
    st = dx.dexel_canonicalize(engine.ctx, v, dx.make_out(2, 1, *o), ws, None, dx.DEXEL_FLAG_SYNC)
    assert st == dx.DEXEL_ERR_CAPACITY and int(o[2].item()) == 2
