"""ctypes binding of libdexel (see include/dexel.h).

Argument marshalling only: every step of the offset runs in the HIP kernels
of libdexel.so.  Torch tensors provide device memory and streams.  Importing
this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_float, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdexel.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdexel.so is not built ({LIB_PATH}); run __graft_entry__.build()")

lib = ctypes.CDLL(LIB_PATH)

# status codes and ops (mirror dexel.h)
DEXEL_OK = 0
DEXEL_ERR_INVALID = -1
DEXEL_ERR_NOT_CANONICAL = -2
DEXEL_ERR_CAPACITY = -3
DEXEL_ERR_WORKSPACE = -4
DEXEL_ERR_HIP = -5
DEXEL_ERR_UNSUPPORTED = -6
DEXEL_DILATE, DEXEL_ERODE, DEXEL_OPEN, DEXEL_CLOSE = 0, 1, 2, 3
OPS = {"dilate": DEXEL_DILATE, "erode": DEXEL_ERODE, "open": DEXEL_OPEN, "close": DEXEL_CLOSE}
DEXEL_FLAG_SYNC = 1
DEXEL_FLAG_VALIDATE = 2
DEXEL_FLAG_RAYS_X = 4
DEXEL_FLAG_RAYS_Y = 8
DEXEL_FLAG_GENERAL = 16
DEXEL_NOALLOC_SCRATCH_BYTES = 256 << 20
RAY_FLAGS = {"x": DEXEL_FLAG_RAYS_X, "y": DEXEL_FLAG_RAYS_Y, "z": 0}
DEXEL_CSG_UNION, DEXEL_CSG_INTERSECT, DEXEL_CSG_DIFFERENCE = 0, 1, 2
CSG_OPS = {"union": DEXEL_CSG_UNION, "intersect": DEXEL_CSG_INTERSECT,
           "difference": DEXEL_CSG_DIFFERENCE}
DEXEL_PRIM_BALL, DEXEL_PRIM_BOX = 0, 1


class dexel_grid_view(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nseg", c_int64),
                ("col_ptr", c_void_p), ("z", c_void_p)]


class dexel_grid_out(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("cap_seg", c_int64),
                ("col_ptr", c_void_p), ("z", c_void_p),
                ("nseg_out", c_void_p), ("status", c_void_p)]


class dexel_batch_item(ctypes.Structure):
    _fields_ = [("in_", dexel_grid_view), ("r", c_float), ("op", c_int32),
                ("out", dexel_grid_out)]


_P = ctypes.POINTER
lib.dexel_ctx_create.argtypes = [c_int, _P(c_void_p)]
lib.dexel_ctx_create.restype = c_int
lib.dexel_ctx_destroy.argtypes = [c_void_p]
lib.dexel_ctx_destroy.restype = None
lib.dexel_workspace_size.argtypes = [c_void_p, _P(dexel_grid_view), c_float, c_int32, c_int64,
                                     _P(c_size_t)]
lib.dexel_workspace_size.restype = c_int
lib.dexel_offset_noalloc.argtypes = [c_void_p, _P(dexel_grid_view), c_float, c_int32, _P(dexel_grid_out),
                                     c_void_p, c_uint32]
lib.dexel_offset_noalloc.restype = c_int
lib.dexel_workspace_need.argtypes = [c_void_p, c_void_p, _P(c_int64)]
lib.dexel_workspace_need.restype = c_int
for _name in ("dexel_dilate", "dexel_erode"):
    getattr(lib, _name).argtypes = [c_void_p, _P(dexel_grid_view), c_float, _P(dexel_grid_out),
                                    c_void_p, c_size_t, c_void_p, c_uint32]
    getattr(lib, _name).restype = c_int
lib.dexel_offset.argtypes = [c_void_p, _P(dexel_grid_view), c_float, c_int32, _P(dexel_grid_out),
                             c_void_p, c_size_t, c_void_p, c_uint32]
lib.dexel_offset.restype = c_int
lib.dexel_batch_workspace_size.argtypes = [c_void_p, c_int32, _P(dexel_batch_item), c_int64,
                                           _P(c_size_t)]
lib.dexel_batch_workspace_size.restype = c_int
lib.dexel_batch_offset.argtypes = [c_void_p, c_int32, _P(dexel_batch_item), c_void_p, c_size_t,
                                   c_void_p, c_uint32]
lib.dexel_batch_offset.restype = c_int
lib.dexel_csg_workspace_size.argtypes = [c_void_p, _P(dexel_grid_view), _P(c_size_t)]
lib.dexel_csg_workspace_size.restype = c_int
lib.dexel_csg.argtypes = [c_void_p, _P(dexel_grid_view), _P(dexel_grid_view), c_int32,
                          _P(dexel_grid_out), c_void_p, c_size_t, c_void_p, ctypes.c_uint32]
lib.dexel_csg.restype = c_int
lib.dexel_dexelize_workspace_size.argtypes = [c_void_p, c_int32, c_int32, _P(c_size_t)]
lib.dexel_dexelize_workspace_size.restype = c_int
lib.dexel_dexelize.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_int32, _P(dexel_grid_out),
                               c_void_p, c_size_t, c_void_p, ctypes.c_uint32]
lib.dexel_dexelize.restype = c_int
lib.dexel_canonicalize_workspace_size.argtypes = [c_void_p, _P(dexel_grid_view), _P(c_size_t)]
lib.dexel_canonicalize_workspace_size.restype = c_int
lib.dexel_canonicalize.argtypes = [c_void_p, _P(dexel_grid_view), _P(dexel_grid_out), c_void_p, c_size_t,
                                   c_void_p, ctypes.c_uint32]
lib.dexel_canonicalize.restype = c_int
lib.dexel_profile_enable.argtypes = [c_void_p, c_int]
lib.dexel_profile_enable.restype = c_int
lib.dexel_profile_read.argtypes = [c_void_p, _P(ctypes.c_double), _P(c_int64), c_int]
lib.dexel_profile_read.restype = c_int
lib.dexel_workspace_stats.argtypes = [c_void_p, c_void_p, _P(c_int64)]
lib.dexel_workspace_stats.restype = c_int
lib.dexel_set_variant.argtypes = [c_void_p, c_int]
lib.dexel_set_variant.restype = c_int
lib.dexel_autotune.argtypes = [c_void_p, c_int32, _P(dexel_batch_item), c_void_p, c_size_t, c_void_p,
                               c_int32, _P(c_int32), _P(ctypes.c_float)]
lib.dexel_autotune.restype = c_int
lib.dexel_status_string.argtypes = [c_int]
lib.dexel_status_string.restype = ctypes.c_char_p
lib.dexel_last_error.argtypes = [c_void_p]
lib.dexel_last_error.restype = ctypes.c_char_p

EXPORTED = ["dexel_ctx_create", "dexel_ctx_destroy", "dexel_workspace_size",
            "dexel_workspace_need", "dexel_dilate", "dexel_erode", "dexel_offset", "dexel_offset_noalloc",
            "dexel_batch_workspace_size", "dexel_batch_offset", "dexel_profile_enable",
            "dexel_profile_read", "dexel_workspace_stats", "dexel_set_variant",
            "dexel_autotune", "dexel_status_string", "dexel_last_error",
            "dexel_csg_workspace_size", "dexel_csg", "dexel_dexelize_workspace_size",
            "dexel_dexelize", "dexel_canonicalize_workspace_size", "dexel_canonicalize"]
NVARIANT = 4
NPROF = 15
PROFILE_STAGES = ["column_gaps", "direct", "thin_erosion", "chord_extremes", "row_offset", "row_offset_replay",
                  "gap_cut", "neighbour", "neighbour_replay", "seeds", "seeds_replay", "y_union",
                  "y_union_replay", "result_scan", "compact"]
# main HIP kernel of each profiled group (as rocprofv3 names it)
PROFILE_KERNELS = ["k_col_gaps", "k_direct", "k_thin_erode", "k_solid_dilate", "k_row_offset", "k_row_offset_fb",
                   "k_gap_cut", "k_neighbour", "k_neighbour_fb", "k_seeds", "k_seeds_fb", "k_union",
                   "k_union_fb", "k_scan", "k_copy_out"]


class DexelError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{dexel_status_string(status)} ({status}) {msg}".strip())


def dexel_status_string(status: int) -> str:
    return lib.dexel_status_string(int(status)).decode()


def dexel_last_error(ctx) -> str:
    return lib.dexel_last_error(ctx).decode()


def dexel_ctx_create(device: int = 0):
    h = c_void_p()
    st = lib.dexel_ctx_create(int(device), ctypes.byref(h))
    if st != DEXEL_OK:
        raise DexelError(st, "dexel_ctx_create")
    return h


def dexel_ctx_destroy(ctx) -> None:
    lib.dexel_ctx_destroy(ctx)


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def make_view(nx: int, ny: int, col_ptr: torch.Tensor, z: torch.Tensor, nseg: int | None = None):
    if nseg is None:
        nseg = z.numel() // 2
    return dexel_grid_view(int(nx), int(ny), int(nseg), _ptr(col_ptr), _ptr(z))


def make_out(nx, ny, col_ptr, z, nseg_out, status):
    return dexel_grid_out(int(nx), int(ny), int(z.numel() // 2), _ptr(col_ptr), _ptr(z),
                          _ptr(nseg_out), _ptr(status))


def dexel_workspace_size(ctx, view: dexel_grid_view, r: float, op: int, cap_hint: int = 0) -> int:
    b = c_size_t()
    st = lib.dexel_workspace_size(ctx, ctypes.byref(view), float(r), int(op), int(cap_hint),
                                  ctypes.byref(b))
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return int(b.value)


def dexel_workspace_need(ctx, ws: torch.Tensor) -> int:
    v = c_int64()
    st = lib.dexel_workspace_need(ctx, _ptr(ws), ctypes.byref(v))
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return int(v.value)


def dexel_offset_noalloc(ctx, view, r, op, out, stream=None, flags: int = 0) -> int:
    """dexel_offset on the library's static device scratch (allocates nothing)."""
    return lib.dexel_offset_noalloc(ctx, ctypes.byref(view), float(r), int(op), ctypes.byref(out),
                                    _stream_ptr(stream), int(flags))


def dexel_offset(ctx, view, r, op, out, ws: torch.Tensor, stream=None, flags: int = 0) -> int:
    return lib.dexel_offset(ctx, ctypes.byref(view), float(r), int(op), ctypes.byref(out),
                            _ptr(ws), int(ws.numel()), _stream_ptr(stream), int(flags))


def dexel_dilate(ctx, view, r, out, ws, stream=None, flags: int = 0) -> int:
    return lib.dexel_dilate(ctx, ctypes.byref(view), float(r), ctypes.byref(out), _ptr(ws),
                            int(ws.numel()), _stream_ptr(stream), int(flags))


def dexel_erode(ctx, view, r, out, ws, stream=None, flags: int = 0) -> int:
    return lib.dexel_erode(ctx, ctypes.byref(view), float(r), ctypes.byref(out), _ptr(ws),
                           int(ws.numel()), _stream_ptr(stream), int(flags))


def dexel_csg_workspace_size(ctx, view: dexel_grid_view) -> int:
    b = c_size_t()
    st = lib.dexel_csg_workspace_size(ctx, ctypes.byref(view), ctypes.byref(b))
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return int(b.value)


def dexel_csg(ctx, a, b, op, out, ws: torch.Tensor, stream=None, flags: int = 0) -> int:
    return lib.dexel_csg(ctx, ctypes.byref(a), ctypes.byref(b), int(op), ctypes.byref(out), _ptr(ws),
                         int(ws.numel()), _stream_ptr(stream), int(flags))


def dexel_dexelize_workspace_size(ctx, nx: int, ny: int) -> int:
    b = c_size_t()
    st = lib.dexel_dexelize_workspace_size(ctx, int(nx), int(ny), ctypes.byref(b))
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return int(b.value)


def dexel_dexelize(ctx, nx, ny, prims: torch.Tensor, out, ws: torch.Tensor, stream=None,
                   flags: int = 0) -> int:
    """prims: float64 device tensor of shape (n, 7)."""
    n = 0 if prims is None else int(prims.numel() // 7)
    return lib.dexel_dexelize(ctx, int(nx), int(ny), _ptr(prims) if n else None, n,
                              ctypes.byref(out), _ptr(ws), int(ws.numel()), _stream_ptr(stream),
                              int(flags))


def dexel_canonicalize_workspace_size(ctx, view) -> int:
    b = c_size_t()
    st = lib.dexel_canonicalize_workspace_size(ctx, ctypes.byref(view), ctypes.byref(b))
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return int(b.value)


def dexel_canonicalize(ctx, view, out, ws: torch.Tensor, stream=None, flags: int = 0) -> int:
    return lib.dexel_canonicalize(ctx, ctypes.byref(view), ctypes.byref(out), _ptr(ws), int(ws.numel()),
                                  _stream_ptr(stream), int(flags))


def dexel_batch_workspace_size(ctx, items, cap_hint: int = 0) -> int:
    arr = (dexel_batch_item * len(items))(*items)
    b = c_size_t()
    st = lib.dexel_batch_workspace_size(ctx, len(items), arr, int(cap_hint), ctypes.byref(b))
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return int(b.value)


def dexel_batch_offset(ctx, items, ws: torch.Tensor, stream=None, flags: int = 0) -> int:
    arr = (dexel_batch_item * len(items))(*items)
    return lib.dexel_batch_offset(ctx, len(items), arr, _ptr(ws), int(ws.numel()),
                                  _stream_ptr(stream), int(flags))


def dexel_profile_enable(ctx, on: bool = True) -> None:
    st = lib.dexel_profile_enable(ctx, 1 if on else 0)
    if st != DEXEL_OK:
        raise DexelError(st)


def dexel_profile_read(ctx, reset: bool = False):
    """Returns (ms per stage as a list, number of passes)."""
    ms = (ctypes.c_double * NPROF)()
    n = c_int64()
    st = lib.dexel_profile_read(ctx, ms, ctypes.byref(n), 1 if reset else 0)
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return list(ms), int(n.value)


def dexel_workspace_stats(ctx, ws: torch.Tensor) -> dict:
    v = (c_int64 * 8)()
    st = lib.dexel_workspace_stats(ctx, _ptr(ws), v)
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    keys = ["row_offset", "neighbour", "seeds", "result", "arena", "replayed", "need", "nseg_out"]
    return dict(zip(keys, list(v)))


def dexel_set_variant(ctx, variant: int) -> None:
    st = lib.dexel_set_variant(ctx, int(variant))
    if st != DEXEL_OK:
        raise DexelError(st)


def dexel_autotune(ctx, items, ws: torch.Tensor, stream=None, reps: int = 2):
    """Returns (chosen variant, ms per variant)."""
    arr = (dexel_batch_item * len(items))(*items)
    chosen = c_int32()
    ms = (ctypes.c_float * NVARIANT)()
    st = lib.dexel_autotune(ctx, len(items), arr, _ptr(ws), int(ws.numel()), _stream_ptr(stream),
                            int(reps), ctypes.byref(chosen), ms)
    if st != DEXEL_OK:
        raise DexelError(st, dexel_last_error(ctx))
    return int(chosen.value), list(ms)
