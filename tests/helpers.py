"""Test helpers: grid construction, an independent point-sampled membership
test, and the tolerance comparator used for GPU-vs-oracle parity.

Nothing here calls the GPU library or the oracle's internals.
"""
from __future__ import annotations

import math

import numpy as np


class HostGrid:
    def __init__(self, nx, ny, col_ptr, z):
        self.nx, self.ny = int(nx), int(ny)
        self.col_ptr = np.asarray(col_ptr, dtype=np.int64)
        self.z = np.asarray(z, dtype=np.float64).reshape(-1)

    @property
    def nseg(self):
        return int(self.col_ptr[-1])

    def column(self, c):
        return self.z[2 * self.col_ptr[c]: 2 * self.col_ptr[c + 1]].reshape(-1, 2)

    def columns(self):
        return [self.column(c) for c in range(self.nx * self.ny)]


def grid_from_columns(nx, ny, cols):
    """cols: list (column id order) of lists of (lo, hi)."""
    cnt = np.array([len(c) for c in cols], dtype=np.int64)
    col_ptr = np.zeros(nx * ny + 1, np.int64)
    np.cumsum(cnt, out=col_ptr[1:])
    z = np.array([v for c in cols for iv in c for v in iv], dtype=np.float64)
    return HostGrid(nx, ny, col_ptr, z)


def random_grid(rng, nx, ny, height, max_per_col=4, p_empty=0.3, f32=True):
    """Canonical random columns (sorted, strictly separated)."""
    cols = []
    for _ in range(nx * ny):
        if rng.random() < p_empty:
            cols.append([])
            continue
        k = int(rng.integers(1, max_per_col + 1))
        pts = np.sort(rng.uniform(0, height, size=2 * k))
        if f32:
            pts = pts.astype(np.float32).astype(np.float64)
        iv = []
        for i in range(k):
            a, b = pts[2 * i], pts[2 * i + 1]
            if iv and a <= iv[-1][1]:
                iv[-1] = (iv[-1][0], max(b, iv[-1][1]))
            else:
                iv.append((a, b))
        cols.append(iv)
    return grid_from_columns(nx, ny, cols)


# ---------------------------------------------------------------------------
# independent membership test by distances (not by chords)
# ---------------------------------------------------------------------------

def _dist_to_intervals(zs, iv):
    """Distance from each sample to the union of closed intervals iv."""
    if len(iv) == 0:
        return np.full(zs.shape, np.inf)
    a = iv[:, 0][None, :]
    b = iv[:, 1][None, :]
    zz = zs[:, None]
    d = np.maximum(np.maximum(a - zz, zz - b), 0.0)
    return d.min(axis=1)


def _dist_to_complement(zs, iv):
    """Distance from each sample to the complement of the union of iv
    (0 outside the intervals)."""
    out = np.zeros(zs.shape)
    for lo, hi in iv:
        inside = (zs >= lo) & (zs <= hi)
        out[inside] = np.minimum(zs[inside] - lo, hi - zs[inside])
    return out


def sampled_membership(grid: HostGrid, r: float, op: str, c: int, zs: np.ndarray) -> np.ndarray:
    """True where the sample (x, y, z) lies in the dilation (any point of the
    shape within distance r) or in the erosion (no point of the in-grid
    complement within distance r) of the grid, for output column c."""
    x, y = c % grid.nx, c // grid.nx
    R = int(math.floor(r)) + 1
    best = np.full(zs.shape, np.inf)
    for yy in range(max(0, y - R), min(grid.ny, y + R + 1)):
        for xx in range(max(0, x - R), min(grid.nx, x + R + 1)):
            d2 = (xx - x) ** 2 + (yy - y) ** 2
            iv = grid.column(yy * grid.nx + xx)
            if op == "dilate":
                dz = _dist_to_intervals(zs, iv)
            else:
                dz = _dist_to_complement(zs, iv)
            best = np.minimum(best, d2 + dz * dz)
    if op == "dilate":
        return best <= r * r
    return best > r * r


def intervals_membership(iv, zs):
    m = np.zeros(zs.shape, bool)
    for lo, hi in iv:
        m |= (zs >= lo) & (zs <= hi)
    return m


def near_endpoint(iv, zs, eps=1e-9):
    m = np.zeros(zs.shape, bool)
    for lo, hi in iv:
        m |= (np.abs(zs - lo) < eps) | (np.abs(zs - hi) < eps)
    return m


# ---------------------------------------------------------------------------
# comparator: GPU (float32) against oracle (float64)
# ---------------------------------------------------------------------------

def ulp32(v):
    v = np.abs(np.asarray(v, dtype=np.float64))
    v32 = np.minimum(v, 3.0e38).astype(np.float32)
    return (np.nextafter(v32, np.float32(np.inf)) - v32).astype(np.float64)


def tau(z, r, k=1):
    """Endpoint tolerance: max(1e-5, ulp32(|z| + r)), times the chain length k."""
    return k * np.maximum(1e-5, ulp32(np.abs(z) + r))


def gamma(z, r, k=1):
    """Gap / length tolerance: max(1e-6, 2 ulp32(|z| + r)), times k."""
    return k * np.maximum(1e-6, 2.0 * ulp32(np.abs(z) + r))


def _column_match(O, G, r, k):
    """Monotone matching of endpoint sequences allowing tiny gaps to merge
    and tiny intervals to vanish on either side.  O, G: (n, 2) arrays."""
    eo = O.reshape(-1)
    eg = G.reshape(-1)
    no, ng = eo.size, eg.size
    fin_o = np.where(np.isfinite(eo), eo, 0.0)
    fin_g = np.where(np.isfinite(eg), eg, 0.0)
    to = tau(fin_o, r, k)
    go = gamma(fin_o, r, k)
    gg = gamma(fin_g, r, k)

    def close(i, j):
        a, b = eo[i], eg[j]
        if not (np.isfinite(a) and np.isfinite(b)):
            return a == b
        return abs(a - b) <= to[i]

    def tiny_o(i):  # pair (i, i+1) of O is a tiny interval or a tiny gap
        return i + 1 < no and eo[i + 1] - eo[i] < go[i]

    def tiny_g(j):
        return j + 1 < ng and eg[j + 1] - eg[j] < gg[j]

    seen = set()
    stack = [(0, 0)]
    while stack:
        i, j = stack.pop()
        if (i, j) in seen:
            continue
        seen.add((i, j))
        if i == no and j == ng:
            return True
        # endpoint types alternate lo/hi; parity must agree for a match
        if i < no and j < ng and (i % 2) == (j % 2) and close(i, j):
            stack.append((i + 1, j + 1))
        if tiny_o(i):
            stack.append((i + 2, j))
        if tiny_g(j):
            stack.append((i, j + 2))
    return False


def compare_columns(o_cnt, o_z, g_cnt, g_z, r, k=1, max_report=5):
    """Compare per-column interval lists.  Returns a dict with counts of
    strict passes (same count, all endpoints within tau), tolerant passes,
    failures and the literal 1e-5 pass fraction."""
    o_cnt = np.asarray(o_cnt, dtype=np.int64)
    g_cnt = np.asarray(g_cnt, dtype=np.int64)
    o_z = np.asarray(o_z, dtype=np.float64).reshape(-1, 2)
    g_z = np.asarray(g_z, dtype=np.float64).reshape(-1, 2)
    o_off = np.concatenate([[0], np.cumsum(o_cnt)])
    g_off = np.concatenate([[0], np.cumsum(g_cnt)])
    n = o_cnt.size
    same = o_cnt == g_cnt
    strict = np.zeros(n, bool)
    lit = np.zeros(n, bool)
    if o_z.size and same.any():
        # vectorised check for equal-count columns
        idx_cols = np.flatnonzero(same)
        eq_rows = np.concatenate([np.arange(o_off[c], o_off[c + 1]) for c in idx_cols]) \
            if idx_cols.size else np.zeros(0, np.int64)
        eq_rows_g = np.concatenate([np.arange(g_off[c], g_off[c + 1]) for c in idx_cols]) \
            if idx_cols.size else np.zeros(0, np.int64)
        O = o_z[eq_rows]
        G = g_z[eq_rows_g]
        finite = np.isfinite(O)
        Of = np.where(finite, O, 0.0)
        Gf = np.where(np.isfinite(G), G, 0.0)
        diff = np.abs(Of - Gf)
        okv = np.where(finite, diff <= tau(Of, r, k), O == G)
        okl = np.where(finite, diff <= 1e-5 * k, O == G)
        rowok = okv.all(axis=1)
        rowlit = okl.all(axis=1)
        col_of_row = np.repeat(idx_cols, o_cnt[idx_cols])
        bad_cols = np.unique(col_of_row[~rowok])
        badl_cols = np.unique(col_of_row[~rowlit])
        strict[idx_cols] = True
        strict[bad_cols] = False
        lit[idx_cols] = True
        lit[badl_cols] = False
    elif same.any():
        strict[same] = True
        lit[same] = True
    tolerant = strict.copy()
    fails = []
    for c in np.flatnonzero(~strict):
        O = o_z[o_off[c]:o_off[c + 1]]
        G = g_z[g_off[c]:g_off[c + 1]]
        if _column_match(O, G, r, k):
            tolerant[c] = True
        elif len(fails) < max_report:
            fails.append((int(c), O.tolist(), G.tolist()))
    return {
        "columns": int(n),
        "strict": int(strict.sum()),
        "tolerant": int(tolerant.sum()),
        "failed": int((~tolerant).sum()),
        "literal_1e-5_fraction": float(lit.mean()) if n else 1.0,
        "examples": fails,
    }
