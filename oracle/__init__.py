"""FP64 brute-force oracle for dexel dilation / erosion (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only callers allowed.  Nothing here is
shared with the GPU library, and the GPU library never imports this package.

Definitions follow Chen, Panozzo, Dumas, "Half-Space Power Diagrams and
Discrete Surface Offsets": dilation is the set of points within distance r
of the shape (Sec. 3.1, "Dilation"); erosion is the complement of the
dilated complement (Sec. 3.1, "Erosion"); opening and closing chain the two
(Sec. 4, "Topological Cleaning").  The dilation is evaluated by the paper's
own brute force (Sec. 4, "Baseline Comparison"): every interval emits its
dilated chord into every column within distance r, and all chords are
merged.  The C implementation is in ``oracle.c``.

Two precisions: ``"f64"`` (the reference) and ``"f32model"`` (the same
definition with every chord end rounded once to float32 and the chord
half-width rounded once to float32), which models a float32 evaluation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the mutation tests load a deliberately broken build.
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

MODES = {"f64": 0, "f32model": 1}
OPS = {"dilate": 0, "erode": 1}


def compile_source(src: str, out: str) -> str:
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if os.environ.get("ORACLE_LIB"):
        return LIB_PATH
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        compile_source(src, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_offset.restype = ctypes.c_int64
        lib.oracle_offset.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


class Grid:
    """Dexel grid in float64: column pointers and (z_in, z_out) pairs."""

    def __init__(self, nx, ny, col_ptr, z):
        self.nx, self.ny = int(nx), int(ny)
        self.col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
        self.z = np.ascontiguousarray(z, dtype=np.float64)

    @classmethod
    def from_any(cls, g):
        return cls(g.nx, g.ny, g.col_ptr, np.asarray(g.z, dtype=np.float64))

    def column(self, c):
        return self.z[2 * self.col_ptr[c]: 2 * self.col_ptr[c + 1]].reshape(-1, 2)

    @property
    def nseg(self):
        return int(self.col_ptr[-1])


def offset_columns(grid, r: float, op: str = "dilate", mode: str = "f64", cols=None):
    """Offset of the requested output columns (all columns if ``cols`` is None).

    Returns ``(counts int64[len(cols)], z float64[2*sum])``.  ``r`` is rounded
    to float32 first, as the GPU library receives it.
    """
    g = grid if isinstance(grid, Grid) else Grid.from_any(grid)
    lib = _load()
    if cols is None:
        cols = np.arange(g.nx * g.ny, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    cnt = np.zeros(cols.size, np.int64)
    rr = float(np.float32(r))
    cap = max(16, 2 * g.nseg + 2 * cols.size)
    while True:
        out = np.empty(2 * cap, np.float64)
        tot = lib.oracle_offset(g.nx, g.ny, g.col_ptr.ctypes.data, g.z.ctypes.data, rr,
                                MODES[mode], OPS[op], cols.size, cols.ctypes.data,
                                cnt.ctypes.data, out.ctypes.data, cap)
        if tot < 0:
            raise ValueError("oracle: invalid arguments")
        if tot <= cap:
            return cnt, out[: 2 * tot]
        cap = int(tot)


def offset(grid, r: float, op: str = "dilate", mode: str = "f64") -> Grid:
    """Offset of a whole grid; returns a float64 ``Grid``."""
    g = grid if isinstance(grid, Grid) else Grid.from_any(grid)
    cnt, z = offset_columns(g, r, op, mode)
    col_ptr = np.zeros(g.nx * g.ny + 1, np.int64)
    np.cumsum(cnt, out=col_ptr[1:])
    return Grid(g.nx, g.ny, col_ptr, z)


def _to_f32_grid(g: Grid) -> Grid:
    """Round every endpoint to float32 (intervals stay as computed)."""
    return Grid(g.nx, g.ny, g.col_ptr, g.z.astype(np.float32).astype(np.float64))


def chain(grid, r: float, ops, mode: str = "f64") -> Grid:
    """Apply ``ops`` (e.g. ["dilate", "erode"] = closing) in sequence.

    In ``f64`` mode the intermediate is kept in float64 (no rounding); in
    ``f32model`` mode it is rounded to float32 between operations.
    """
    g = grid if isinstance(grid, Grid) else Grid.from_any(grid)
    for op in ops:
        g = offset(g, r, op, mode)
        if mode == "f32model":
            g = _to_f32_grid(g)
    return g


CHAINS = {"dilate": ["dilate"], "erode": ["erode"], "close": ["dilate", "erode"],
          "open": ["erode", "dilate"]}


def run(grid, r: float, op: str, mode: str = "f64") -> Grid:
    return chain(grid, r, CHAINS[op], mode)


def region_chain(grid, r: float, op: str, cols, mode: str = "f64"):
    """Chained op evaluated only on the requested columns.

    For a chain of k operations the first operation is evaluated on every
    column within k-1 stencil radii of a requested column, the next on the
    columns within k-2 radii, and so on; columns outside the neighbourhood
    are never read by the requested outputs.
    """
    g = grid if isinstance(grid, Grid) else Grid.from_any(grid)
    ops = CHAINS[op]
    R = int(np.floor(np.float32(r)))
    cols = np.unique(np.asarray(cols, dtype=np.int64))
    xs, ys = cols % g.nx, cols // g.nx
    need = []
    for k in range(len(ops)):
        grow = R * (len(ops) - 1 - k)
        mask = np.zeros((g.ny, g.nx), bool)
        for x, y in zip(xs, ys):
            mask[max(0, y - grow): y + grow + 1, max(0, x - grow): x + grow + 1] = True
        need.append(np.flatnonzero(mask.ravel()))
    cur = g
    for k, op1 in enumerate(ops):
        c = need[k]
        cnt, z = offset_columns(cur, r, op1, mode, cols=c)
        full = np.zeros(g.nx * g.ny, np.int64)
        full[c] = cnt
        col_ptr = np.zeros(g.nx * g.ny + 1, np.int64)
        np.cumsum(full, out=col_ptr[1:])
        # offset_columns returns outputs in request order; c is sorted so
        # request order equals column order.
        cur = Grid(g.nx, g.ny, col_ptr, z)
        if mode == "f32model":
            cur = _to_f32_grid(cur)
    cnt = np.diff(cur.col_ptr)[cols]
    z = np.concatenate([cur.column(c).ravel() for c in cols]) if cols.size else np.zeros(0)
    return cnt, z
