"""Seeded generators of dexel grids (CSR: int64 column pointers, float32 pairs).

Column id = y * nx + x (x fastest).  Rays go through cell centres
(x + 1/2, y + 1/2); z is continuous.  Every generator builds float64
intervals, rounds them to the nearest float32 and re-canonicalises them
(sorted, z_in <= z_out, touching or overlapping intervals merged), so every
grid these functions return is a valid canonical dexel buffer.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

GENERATOR_VERSION = 1


@dataclass
class DexelGrid:
    nx: int
    ny: int
    col_ptr: np.ndarray  # int64 [nx*ny + 1]
    z: np.ndarray        # float32 [2 * nseg], (z_in, z_out) pairs
    meta: dict = field(default_factory=dict)

    @property
    def nseg(self) -> int:
        return int(self.col_ptr[-1])

    @property
    def ncols(self) -> int:
        return self.nx * self.ny

    def column(self, x: int, y: int) -> np.ndarray:
        c = y * self.nx + x
        return self.z[2 * self.col_ptr[c]: 2 * self.col_ptr[c + 1]].reshape(-1, 2)

    def stats(self) -> dict:
        cnt = np.diff(self.col_ptr)
        return {
            "nx": self.nx, "ny": self.ny, "nseg": self.nseg,
            "mean_segs_per_col": float(cnt.mean()) if cnt.size else 0.0,
            "p95_segs_per_col": float(np.percentile(cnt, 95)) if cnt.size else 0.0,
            "max_segs_per_col": int(cnt.max()) if cnt.size else 0,
        }


# ---------------------------------------------------------------------------
# canonicalisation of raw float64 intervals
# ---------------------------------------------------------------------------

def _ordered_u32(f32: np.ndarray) -> np.ndarray:
    """Map float32 values to uint32 keys with the same total order."""
    b = (f32 + np.float32(0.0)).view(np.uint32)  # -0.0 -> +0.0
    neg = (b >> np.uint32(31)).astype(bool)
    return np.where(neg, ~b, b | np.uint32(0x80000000)).astype(np.uint32)


def canonical_csr(cols: np.ndarray, lo: np.ndarray, hi: np.ndarray, ncols: int):
    """Round float64 intervals to float32 and merge them per column.

    Intervals whose float32 images overlap or touch are merged.  Returns
    ``(col_ptr int64[ncols+1], z float32[2n])``.
    """
    cols = np.asarray(cols, dtype=np.int64)
    lo32 = np.asarray(lo, dtype=np.float64).astype(np.float32)
    hi32 = np.asarray(hi, dtype=np.float64).astype(np.float32)
    if cols.size == 0:
        return np.zeros(ncols + 1, np.int64), np.zeros(0, np.float32)
    if np.any(hi32 < lo32) or not (np.all(np.isfinite(lo32)) and np.all(np.isfinite(hi32))):
        raise ValueError("intervals must be finite with lo <= hi")
    klo = (cols.astype(np.uint64) << np.uint64(32)) | _ordered_u32(lo32).astype(np.uint64)
    khi = (cols.astype(np.uint64) << np.uint64(32)) | _ordered_u32(hi32).astype(np.uint64)
    order = np.argsort(klo, kind="stable")
    klo, khi = klo[order], khi[order]
    lo32, hi32, cols = lo32[order], hi32[order], cols[order]
    run = np.maximum.accumulate(khi)
    start = np.ones(cols.size, dtype=bool)
    start[1:] = klo[1:] > run[:-1]
    gidx = np.flatnonzero(start)
    glo = lo32[gidx]
    ghi = np.maximum.reduceat(hi32, gidx)
    gcol = cols[gidx]
    counts = np.bincount(gcol, minlength=ncols).astype(np.int64)
    col_ptr = np.zeros(ncols + 1, np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    z = np.empty(2 * gidx.size, np.float32)
    z[0::2] = glo
    z[1::2] = ghi
    return col_ptr, z


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------

def _sphere_chords(nx, ny, centres, radii, strict=True):
    """Chords of balls along z-rays through cell centres (float64)."""
    cols, lo, hi = [], [], []
    for (cx, cy, cz), R in zip(centres, radii):
        x0 = max(0, int(math.floor(cx - R - 1)))
        x1 = min(nx, int(math.ceil(cx + R + 1)))
        y0 = max(0, int(math.floor(cy - R - 1)))
        y1 = min(ny, int(math.ceil(cy + R + 1)))
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1, dtype=np.float64) + 0.5
        ys = np.arange(y0, y1, dtype=np.float64) + 0.5
        X, Y = np.meshgrid(xs, ys)
        rho2 = (X - cx) ** 2 + (Y - cy) ** 2
        m = rho2 < R * R if strict else rho2 <= R * R
        if not m.any():
            continue
        h = np.sqrt(R * R - rho2[m])
        ix = (X[m] - 0.5).astype(np.int64)
        iy = (Y[m] - 0.5).astype(np.int64)
        cols.append(iy * nx + ix)
        lo.append(cz - h)
        hi.append(cz + h)
    return cols, lo, hi


def _box_chords(nx, ny, lo3, hi3):
    """Boxes [lo3, hi3] sampled along z-rays through cell centres."""
    cols, lo, hi = [], [], []
    for (ax, ay, az), (bx, by, bz) in zip(lo3, hi3):
        x0 = max(0, int(math.ceil(ax - 0.5)))
        x1 = min(nx, int(math.floor(bx - 0.5)) + 1)
        y0 = max(0, int(math.ceil(ay - 0.5)))
        y1 = min(ny, int(math.floor(by - 0.5)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1, dtype=np.int64)
        ys = np.arange(y0, y1, dtype=np.int64)
        X, Y = np.meshgrid(xs, ys)
        c = (Y * nx + X).ravel()
        cols.append(c)
        lo.append(np.full(c.size, az))
        hi.append(np.full(c.size, bz))
    return cols, lo, hi


def _assemble(nx, ny, parts, meta):
    cols, lo, hi = parts
    if cols:
        cols = np.concatenate(cols)
        lo = np.concatenate(lo)
        hi = np.concatenate(hi)
    else:
        cols = np.zeros(0, np.int64)
        lo = hi = np.zeros(0)
    col_ptr, z = canonical_csr(cols, lo, hi, nx * ny)
    g = DexelGrid(nx, ny, col_ptr, z, dict(meta))
    g.meta.update(g.stats())
    g.meta["generator_version"] = GENERATOR_VERSION
    return g


def spheres_grid(seed: int, n: int = 64, count: int = 8, rmin: float = 4.0,
                 rmax: float = 12.0) -> DexelGrid:
    """Union of ``count`` balls, radius U[rmin, rmax], centres U[R, n-R]^3."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(rmin, rmax, size=count)
    centres = np.stack([rng.uniform(R, n - R, size=3) for R in radii])
    parts = _sphere_chords(n, n, centres, radii)
    return _assemble(n, n, parts, {"generator": "spheres", "seed": seed, "n": n,
                                   "count": count, "height": n})


def primitives_grid(seed: int, n: int = 512, count: int = 1350, smin: float = 4.0,
                    smax: float = 64.0, height: float | None = None) -> DexelGrid:
    """Union of ``count`` spheres (diameter U[smin,smax]) and axis-aligned
    boxes (edges U[smin,smax] per axis), each with probability 1/2; centres
    U[0,n]^2 x U[0,height].  Footprints are clipped to the grid, z is not."""
    rng = np.random.default_rng(seed)
    height = float(n if height is None else height)
    kind = rng.random(count) < 0.5
    centres = np.column_stack([rng.uniform(0, n, count), rng.uniform(0, n, count),
                               rng.uniform(0, height, count)])
    sizes = rng.uniform(smin, smax, size=(count, 3))
    sc, sr = centres[kind], sizes[kind, 0] / 2.0
    bc, be = centres[~kind], sizes[~kind]
    p1 = _sphere_chords(n, n, sc, sr)
    p2 = _box_chords(n, n, bc - be / 2.0, bc + be / 2.0)
    parts = (p1[0] + p2[0], p1[1] + p2[1], p1[2] + p2[2])
    return _assemble(n, n, parts, {"generator": "primitives", "seed": seed, "n": n,
                                   "count": count, "height": height,
                                   "size_range": [smin, smax]})


def primitive_records(seed: int, n: int = 512, count: int = 1350, smin: float = 4.0,
                      smax: float = 64.0, height: float | None = None) -> np.ndarray:
    """The primitives of ``primitives_grid`` with the same arguments (same
    random draws), as records (kind, a0, a1, a2, b0, b1, b2): kind 0 = ball
    (a = centre, b0 = radius), kind 1 = box (a = low corner, b = high corner)."""
    rng = np.random.default_rng(seed)
    height = float(n if height is None else height)
    kind = rng.random(count) < 0.5
    centres = np.column_stack([rng.uniform(0, n, count), rng.uniform(0, n, count),
                               rng.uniform(0, height, count)])
    sizes = rng.uniform(smin, smax, size=(count, 3))
    rec = np.zeros((count, 7), np.float64)
    rec[kind, 0] = 0.0
    rec[kind, 1:4] = centres[kind]
    rec[kind, 4] = sizes[kind, 0] / 2.0
    rec[~kind, 0] = 1.0
    rec[~kind, 1:4] = centres[~kind] - sizes[~kind] / 2.0
    rec[~kind, 4:7] = centres[~kind] + sizes[~kind] / 2.0
    return rec


def _gyroid_rows(args):
    """Canonical CSR of gyroid rows [yb, ye) (worker for gyroid_grid)."""
    n, H, period, t, ph, yb, ye = args
    k = 2.0 * math.pi / period
    nper = int(math.ceil(H / period)) + 4
    xs = np.arange(n, dtype=np.float64)
    X, Y = np.meshgrid(xs + 0.5 + ph[0], np.arange(yb, ye, dtype=np.float64) + 0.5 + ph[1])
    X, Y = X.ravel(), Y.ravel()
    cid = np.arange((ye - yb) * n, dtype=np.int64)
    A = np.sin(k * X) * np.cos(k * Y)
    sy, cx = np.sin(k * Y), np.cos(k * X)
    M = np.sqrt(sy * sy + cx * cx)
    theta = np.arctan2(cx, sy)
    flat = M < 1e-12
    Ms = np.where(flat, 1.0, M)
    ulo = np.maximum(-1.0, (-t - A) / Ms)
    uhi = np.minimum(1.0, (t - A) / Ms)
    some = (ulo <= uhi) & ~flat
    full_flat = flat & (np.abs(A) <= t)
    alpha = np.arccos(np.clip(uhi, -1.0, 1.0))
    beta = np.arccos(np.clip(ulo, -1.0, 1.0))
    lo_clip = uhi >= 1.0   # alpha == 0: arcs centred at 2 pi m
    hi_clip = ulo <= -1.0  # beta == pi: arcs centred at 2 pi m + pi
    # phi = k (z + ph_z) - theta ; z = (phi + theta) / k - ph_z
    phi0 = k * ph[2] - theta
    m0 = np.floor(phi0 / (2 * math.pi)) - 2
    ms = m0[:, None] + np.arange(nper + 2)[None, :]
    base = 2 * math.pi * ms
    a_, b_ = alpha[:, None], beta[:, None]
    full = (some & lo_clip & hi_clip) | full_flat
    c1 = some & lo_clip & ~hi_clip
    c2 = some & hi_clip & ~lo_clip
    c3 = some & ~lo_clip & ~hi_clip
    segs = [(c1, base - b_, base + b_), (c2, base + a_, base + 2 * math.pi - a_),
            (c3, base + a_, base + b_), (c3, base + 2 * math.pi - b_, base + 2 * math.pi - a_)]
    th = theta[:, None]
    cols_all, lo_all, hi_all = [], [], []
    for mask, plo, phi_hi in segs:
        if not mask.any():
            continue
        zl = (plo[mask] + th[mask]) / k - ph[2]
        zh = (phi_hi[mask] + th[mask]) / k - ph[2]
        cc = np.broadcast_to(cid[mask][:, None], zl.shape)
        zl = np.maximum(zl, 0.0)
        zh = np.minimum(zh, H)
        keep = zl < zh
        cols_all.append(cc[keep])
        lo_all.append(zl[keep])
        hi_all.append(zh[keep])
    if full.any():
        cols_all.append(cid[full])
        lo_all.append(np.zeros(int(full.sum())))
        hi_all.append(np.full(int(full.sum()), H))
    if cols_all:
        cols = np.concatenate(cols_all)
        lo = np.concatenate(lo_all)
        hi = np.concatenate(hi_all)
    else:
        cols = np.zeros(0, np.int64)
        lo = hi = np.zeros(0)
    col_ptr, z = canonical_csr(cols, lo, hi, (ye - yb) * n)
    return np.diff(col_ptr).astype(np.int32), z


def gyroid_grid(seed: int, n: int = 2048, height: float | None = None,
                period: float = 64.0, t: float = 0.225,
                rows: tuple[int, int] | None = None, workers: int | None = None) -> DexelGrid:
    """Thin-walled gyroid lattice {|f| <= t}, f = sin kX cos kY + sin kY cos kZ
    + sin kZ cos kX, k = 2 pi / period, with seeded phase shifts, sliced in
    closed form along each z-ray and clipped to z in [0, height].

    Along a ray f = A + M cos(kZ - theta), A = sin kX cos kY,
    M = sqrt(sin^2 kY + cos^2 kX), theta = atan2(cos kX, sin kY).
    ``rows`` restricts generation to y in [rows[0], rows[1]) (same values as
    the full grid there; the returned grid then has ny = rows[1] - rows[0]).
    Rows are generated in independent chunks, in parallel threads for large
    grids (numpy releases the GIL in its array kernels).  No process is
    forked: callers may already hold GPU state, which a forked child must
    not inherit.
    """
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, period, size=3)
    H = float(n if height is None else height)
    y0, y1 = (0, n) if rows is None else rows
    chunk = max(1, (1 << 18) // max(1, n))
    jobs = [(n, H, period, t, ph, yb, min(y1, yb + chunk)) for yb in range(y0, y1, chunk)]
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if len(jobs) >= 8 else 1
    if workers > 1:
        with ThreadPoolExecutor(workers) as pool:
            parts = list(pool.map(_gyroid_rows, jobs))
    else:
        parts = [_gyroid_rows(j) for j in jobs]
    counts = np.concatenate([p[0] for p in parts]).astype(np.int64)
    col_ptr = np.zeros(counts.size + 1, np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    z = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.float32)
    g = DexelGrid(n, y1 - y0, col_ptr, z, {"generator": "gyroid", "seed": seed, "n": n,
                                           "height": H, "period": period, "wall_t": t,
                                           "phase": ph.tolist(), "rows": [y0, y1]})
    g.meta.update(g.stats())
    g.meta["generator_version"] = GENERATOR_VERSION
    return g


# ---------------------------------------------------------------------------
# the five workload configurations
# ---------------------------------------------------------------------------

CONFIGS = {
    "c1": dict(desc="plain dilation, 64x64, 8 random spheres R~U[4,12], r=3", radii=[3.0],
               ops=["dilate"]),
    "c2": dict(desc="plain dilation and erosion, 512x512, 1350 spheres/boxes sizes U[4,64]",
               radii=[2.0, 8.0, 32.0], ops=["dilate", "erode"]),
    "c2lit": dict(desc="as c2 with 200 primitives", radii=[2.0, 8.0, 32.0],
                  ops=["dilate", "erode"]),
    "c3": dict(desc="closing of a 2048x2048 gyroid lattice (period 64, wall ~3 voxels), r=16",
               radii=[16.0], ops=["close"]),
}


def config_grid(name: str, seed: int = 0, **kw) -> DexelGrid:
    if name == "c1":
        return spheres_grid(seed, **kw)
    if name == "c2":
        return primitives_grid(seed, **kw)
    if name == "c2lit":
        return primitives_grid(seed, count=200, **kw)
    if name == "c3":
        return gyroid_grid(seed, **kw)
    raise KeyError(name)


def batch_shapes(seed: int = 0, count: int = 64, smin: int = 128, smax: int = 1024):
    """``count`` shapes: side log-uniform in [smin, smax], 20..300 primitives
    scaled by side/512, per-shape radius U[2, 32] (non-integer)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        s = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        nprim = int(rng.integers(20, 301))
        r = float(rng.uniform(2.0, 32.0))
        sub = int(rng.integers(0, 2**31 - 1))
        scale = s / 512.0
        g = primitives_grid(sub, n=s, count=nprim, smin=4.0 * scale, smax=64.0 * scale,
                            height=float(s))
        g.meta["r"] = r
        out.append((g, r))
    return out


def serving_stream(seed: int, count: int, rate: float, smin: int = 256, smax: int = 2048,
                   rmin: float = 1.0, rmax: float = 24.0, chain_p: float = 0.3):
    """Poisson request stream: (arrival_s, shape spec, op, r, chain flag).

    Shapes are described by generator arguments (not materialised here) so a
    server can build them lazily; half are primitive soups, half gyroids with
    a random phase.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        s = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        if rng.random() < 0.5:
            spec = ("primitives", dict(seed=int(rng.integers(0, 2**31 - 1)), n=s,
                                       count=int(rng.integers(20, 301)),
                                       smin=4.0 * s / 512, smax=64.0 * s / 512,
                                       height=float(s)))
        else:
            spec = ("gyroid", dict(seed=int(rng.integers(0, 2**31 - 1)), n=s))
        op = ["dilate", "erode", "open", "close"][int(rng.integers(0, 4))]
        r = float(rng.uniform(rmin, rmax))
        chain = bool(rng.random() < chain_p)
        reqs.append(dict(id=i, arrival=t, spec=spec, op=op, r=r, chain=chain))
    return reqs


def build_spec(spec) -> DexelGrid:
    kind, kw = spec
    if kind == "primitives":
        return primitives_grid(**kw)
    if kind == "gyroid":
        return gyroid_grid(**kw)
    raise KeyError(kind)
