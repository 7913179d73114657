"""MI355X dexel offsets: exact dilation / erosion of dexel shapes by a ball.

The computation runs in libdexel.so (HIP kernels for gfx950, C ABI in
include/dexel.h).  This package is the Python binding: ``binding`` holds
the thin ctypes wrappers with the C names; ``Engine`` adds buffer
management (device tensors, workspace reuse, retry on capacity).
"""
from __future__ import annotations

import torch

from .binding import (  # noqa: F401
    DEXEL_CLOSE, DEXEL_DILATE, DEXEL_ERODE, DEXEL_ERR_CAPACITY, DEXEL_ERR_HIP,
    DEXEL_ERR_INVALID, DEXEL_ERR_NOT_CANONICAL, DEXEL_ERR_UNSUPPORTED, DEXEL_ERR_WORKSPACE,
    DEXEL_FLAG_SYNC, DEXEL_FLAG_VALIDATE, DEXEL_FLAG_GENERAL, DEXEL_OK, DEXEL_OPEN, EXPORTED, LIB_PATH, OPS,
    DexelError, dexel_batch_item, dexel_batch_offset, dexel_batch_workspace_size,
    dexel_ctx_create, dexel_ctx_destroy, dexel_dilate, dexel_erode, dexel_grid_out,
    dexel_grid_view, dexel_last_error, dexel_offset, dexel_profile_enable, dexel_profile_read,
    dexel_status_string, dexel_workspace_need, dexel_workspace_size, dexel_workspace_stats,
    make_out, make_view, NPROF, PROFILE_KERNELS, PROFILE_STAGES, NVARIANT, dexel_autotune,
    dexel_set_variant, CSG_OPS, DEXEL_CSG_DIFFERENCE, DEXEL_CSG_INTERSECT, DEXEL_CSG_UNION,
    dexel_csg, dexel_csg_workspace_size, DEXEL_PRIM_BALL, DEXEL_PRIM_BOX, dexel_dexelize,
    dexel_dexelize_workspace_size, DEXEL_FLAG_RAYS_X, DEXEL_FLAG_RAYS_Y, RAY_FLAGS,
    dexel_canonicalize, dexel_canonicalize_workspace_size, dexel_offset_noalloc,
    DEXEL_NOALLOC_SCRATCH_BYTES,
)


class DeviceGrid:
    """A dexel grid resident on the GPU (int64 col_ptr, float32 pairs)."""

    def __init__(self, nx: int, ny: int, col_ptr: torch.Tensor, z: torch.Tensor):
        self.nx, self.ny = int(nx), int(ny)
        self.col_ptr = col_ptr
        self.z = z

    @classmethod
    def from_host(cls, g, device="cuda"):
        cp = torch.as_tensor(g.col_ptr, dtype=torch.int64).to(device)
        z = torch.as_tensor(g.z, dtype=torch.float32).reshape(-1)
        if z.numel() == 0:
            z = torch.zeros(2, dtype=torch.float32)
        return cls(g.nx, g.ny, cp, z.to(device))

    @property
    def nseg(self) -> int:
        return int(self.col_ptr[-1].item())

    def view(self, nseg: int | None = None):
        return make_view(self.nx, self.ny, self.col_ptr, self.z,
                         self.nseg if nseg is None else nseg)

    def to_host(self):
        n = self.nseg
        return (self.col_ptr.cpu().numpy(), self.z[: 2 * n].cpu().numpy())


class Engine:
    """Owns a libdexel context and a reusable workspace on one device."""

    def __init__(self, device: int = 0):
        self.device_index = int(device)
        self.device = torch.device("cuda", self.device_index)
        self.ctx = dexel_ctx_create(self.device_index)
        self._ws = None
        # capacity hint (intervals) for the call offset() or batch_offset()
        # last completed: what it used plus a margin, or 0 (the library's
        # default); Plan and BatchPlan size their workspace with it
        self.last_hint = 0

    def close(self):
        if self.ctx is not None:
            dexel_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int) -> torch.Tensor:
        """The engine's scratch workspace, at least `nbytes` long: one buffer
        that only grows, so a call may run on more capacity than it asked for
        (the library uses all of it).  The caller drops its own reference to
        the old buffer before asking for a larger one, so the two are never
        held at once."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return self._ws

    def _note_hint(self, ws: torch.Tensor, default_cap: int) -> None:
        """Record the capacity hint a Plan or BatchPlan should size its own
        workspace with: what the call just completed really used (read from
        the workspace header), with a quarter's margin for the other kernel
        variants, or 0 (the library's default) when that is enough."""
        need = dexel_workspace_need(self.ctx, ws)
        h = int(need * 1.25) + 1024
        self.last_hint = h if h > default_cap else 0

    def offset(self, grid: DeviceGrid, r: float, op: str = "dilate", stream=None,
               out_cap: int | None = None, validate: bool = False, max_tries: int = 8,
               hint: int = 0, flags: int = 0):
        """Run one op synchronously; returns a new DeviceGrid.  Retries on
        workspace or output capacity; `hint` is the first capacity hint (0:
        the library's default for this input), and each retry starts from
        this call's own need, never from another call's.  `flags` adds
        DEXEL_FLAG_* bits (e.g. DEXEL_FLAG_GENERAL) to the call."""
        code = OPS[op]
        nseg = grid.nseg
        view = grid.view(nseg)
        ncols = grid.nx * grid.ny
        cap = out_cap if out_cap is not None else nseg + ncols + 1024
        flags = int(flags) | DEXEL_FLAG_SYNC | (DEXEL_FLAG_VALIDATE if validate else 0)
        ws = col = z = None
        for _ in range(max_tries):
            nbytes = dexel_workspace_size(self.ctx, view, r, code, hint)
            ws = col = z = None  # the last try's buffers go before the next are made
            ws = self.workspace(nbytes)
            col = torch.empty(ncols + 1, dtype=torch.int64, device=self.device)
            z = torch.empty(2 * max(cap, 1), dtype=torch.float32, device=self.device)
            nout = torch.zeros(1, dtype=torch.int64, device=self.device)
            status = torch.zeros(1, dtype=torch.int32, device=self.device)
            out = make_out(grid.nx, grid.ny, col, z, nout, status)
            st = dexel_offset(self.ctx, view, r, code, out, ws, stream, flags)
            if st == DEXEL_OK:
                self._note_hint(ws, nseg + 2 * ncols + 1024)
                return DeviceGrid(grid.nx, grid.ny, col, z)
            if st == DEXEL_ERR_WORKSPACE:
                need = dexel_workspace_need(self.ctx, ws)
                if need <= 0:
                    raise DexelError(st, dexel_last_error(self.ctx))
                # a call stops at the first stage that runs out, so a later
                # stage may need more than `need`: grow at least 1.5x per try
                base = hint if hint > 0 else nseg + 2 * ncols + 1024
                hint = max(int(need * 1.25) + 1024, base + base // 2)
                continue
            if st == DEXEL_ERR_CAPACITY:
                cap = int(nout.item()) + 1
                continue
            raise DexelError(st, dexel_last_error(self.ctx))
        raise DexelError(DEXEL_ERR_WORKSPACE, "retries exhausted")


    def csg(self, a: DeviceGrid, b: DeviceGrid, op: str, stream=None) -> DeviceGrid:
        """Per-column regularised union / intersection / difference of two
        grids of the same size (dexel_csg), synchronously."""
        code = CSG_OPS[op]
        if (a.nx, a.ny) != (b.nx, b.ny):
            raise ValueError("grids differ in size")
        va, vb = a.view(a.nseg), b.view(b.nseg)
        ncols = a.nx * a.ny
        cap = a.nseg + b.nseg + 1
        ws = self.workspace(dexel_csg_workspace_size(self.ctx, va))
        col = torch.empty(ncols + 1, dtype=torch.int64, device=self.device)
        z = torch.empty(2 * cap, dtype=torch.float32, device=self.device)
        nout = torch.zeros(1, dtype=torch.int64, device=self.device)
        status = torch.zeros(1, dtype=torch.int32, device=self.device)
        out = make_out(a.nx, a.ny, col, z, nout, status)
        st = dexel_csg(self.ctx, va, vb, code, out, ws, stream, DEXEL_FLAG_SYNC)
        if st != DEXEL_OK:
            raise DexelError(st, dexel_last_error(self.ctx))
        return DeviceGrid(a.nx, a.ny, col, z)

    def offset_slices(self, slices, r: float, op: str = "dilate", stream=None):
        """2D offsets of many dexel slices (Sec. 3.2: parallel segments on a
        1D grid, offset by a disk), all in one batched enqueue.  A slice is a
        DeviceGrid with ny == 1: the ball restricted to the slice's plane is
        the disk and there is no other row, so the 3D kernels compute the 2D
        offset exactly.  Returns one DeviceGrid per slice."""
        slices = list(slices)
        for g in slices:
            if g.ny != 1:
                raise ValueError("a slice is an nx x 1 grid")
        return batch_offset(self, slices, [r] * len(slices), [op] * len(slices), stream=stream)

    def dexelize(self, nx: int, ny: int, prims, stream=None, max_tries: int = 4,
                 axis: str = "z") -> DeviceGrid:
        """Dexel grid of the union of balls and boxes (dexel_dexelize).
        prims: (n, 7) records (kind, a0, a1, a2, b0, b1, b2), host or device.
        axis: the rays' direction; "x" makes an nx x ny grid over (y, z),
        "y" one over (z, x)."""
        flags = DEXEL_FLAG_SYNC | RAY_FLAGS[axis]
        p = torch.as_tensor(prims, dtype=torch.float64).reshape(-1, 7).to(self.device).contiguous()
        ncols = int(nx) * int(ny)
        ws = self.workspace(dexel_dexelize_workspace_size(self.ctx, nx, ny))
        cap = max(1024, 2 * ncols)
        for _ in range(max_tries):
            col = torch.empty(ncols + 1, dtype=torch.int64, device=self.device)
            z = torch.empty(2 * cap, dtype=torch.float32, device=self.device)
            nout = torch.zeros(1, dtype=torch.int64, device=self.device)
            status = torch.zeros(1, dtype=torch.int32, device=self.device)
            out = make_out(nx, ny, col, z, nout, status)
            st = dexel_dexelize(self.ctx, nx, ny, p, out, ws, stream, flags)
            if st == DEXEL_OK:
                return DeviceGrid(nx, ny, col, z)
            if st == DEXEL_ERR_CAPACITY:
                cap = int(nout.item()) + 1
                continue
            raise DexelError(st, dexel_last_error(self.ctx))
        raise DexelError(DEXEL_ERR_CAPACITY, "retries exhausted")

    def canonicalize(self, nx: int, ny: int, col_ptr, z, stream=None) -> DeviceGrid:
        """Canonical grid (per column: sorted, overlapping or touching
        intervals joined) from columns whose closed intervals come in any
        order (dexel_canonicalize).  col_ptr: int64[nx*ny+1]; z: float32
        pairs; host or device."""
        cp = torch.as_tensor(col_ptr, dtype=torch.int64).reshape(-1).to(self.device).contiguous()
        zz = torch.as_tensor(z, dtype=torch.float32).reshape(-1).to(self.device).contiguous()
        nseg = zz.numel() // 2
        if zz.numel() == 0:
            zz = torch.zeros(2, dtype=torch.float32, device=self.device)
        view = make_view(nx, ny, cp, zz, nseg)
        ws = self.workspace(dexel_canonicalize_workspace_size(self.ctx, view))
        col = torch.empty(int(nx) * int(ny) + 1, dtype=torch.int64, device=self.device)
        out_z = torch.empty(2 * max(nseg, 1), dtype=torch.float32, device=self.device)
        nout = torch.zeros(1, dtype=torch.int64, device=self.device)
        status = torch.zeros(1, dtype=torch.int32, device=self.device)
        out = make_out(nx, ny, col, out_z, nout, status)
        st = dexel_canonicalize(self.ctx, view, out, ws, stream, DEXEL_FLAG_SYNC)
        if st != DEXEL_OK:
            raise DexelError(st, dexel_last_error(self.ctx))
        return DeviceGrid(nx, ny, col, out_z)

    def tridexel(self, dims, prims, stream=None) -> dict:
        """The solid sampled by rays along each of the three axes (the dexel
        structures in three orthogonal directions suggested in the "Limitations"
        paragraph of Sec. 4 and in Sec. 5).  dims = (n0, n1, n2) cells along x, y, z.  Returns
        {"x": n1 x n2 grid over (y, z), "y": n2 x n0 grid over (z, x),
        "z": n0 x n1 grid over (x, y)}."""
        n0, n1, n2 = (int(d) for d in dims)
        return {"x": self.dexelize(n1, n2, prims, stream, axis="x"),
                "y": self.dexelize(n2, n0, prims, stream, axis="y"),
                "z": self.dexelize(n0, n1, prims, stream, axis="z")}

    def tridexel_offset(self, tri: dict, r: float, op: str = "dilate", stream=None) -> dict:
        """Offset of each of the three structures by the same ball, in one
        batched enqueue.  The ball looks the same along every axis, so each
        direction is the method applied to that direction's grid."""
        keys = ("x", "y", "z")
        outs = batch_offset(self, [tri[k] for k in keys], [r] * 3, [op] * 3, stream=stream)
        return dict(zip(keys, outs))

    def shell(self, grid: DeviceGrid, r: float) -> DeviceGrid:
        """Shell of thickness about 2r around the surface: the dilation minus
        the erosion (Sec. 4, "3D Printing"), three library calls on the device."""
        d = self.offset(grid, r, "dilate")
        e = self.offset(grid, r, "erode")
        return self.csg(d, e, "difference")


class Plan:
    """A pre-sized offset call for repeated asynchronous enqueues.

    Construction runs the op once synchronously (learning the workspace and
    output sizes), then keeps the output buffers, its own workspace and the
    call arguments for its lifetime, so that an enqueue (or a captured graph
    replaying one) never writes into memory another call may reallocate.
    ``enqueue`` issues the call on a stream without synchronising;
    ``status()`` reads the device status of the last call.  Enqueues of one
    plan on two streams that may overlap race on its workspace: order them.
    """

    def __init__(self, engine: "Engine", grid: DeviceGrid, r: float, op: str):
        self.engine, self.grid, self.r, self.op = engine, grid, float(r), op
        self.code = OPS[op]
        res = engine.offset(grid, r, op)
        self.nseg_out = res.nseg
        self.nseg_in = grid.nseg
        self.view = grid.view(self.nseg_in)
        ncols = grid.nx * grid.ny
        dev = engine.device
        self.col = torch.empty(ncols + 1, dtype=torch.int64, device=dev)
        self.z = torch.empty(2 * max(self.nseg_out, 1), dtype=torch.float32, device=dev)
        self.nout = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status_t = torch.zeros(1, dtype=torch.int32, device=dev)
        self.out = make_out(grid.nx, grid.ny, self.col, self.z, self.nout, self.status_t)
        self.ws_bytes = dexel_workspace_size(engine.ctx, self.view, self.r, self.code,
                                             engine.last_hint)
        self.ws = torch.empty(int(self.ws_bytes), dtype=torch.uint8, device=dev)

    def enqueue(self, stream=None, flags: int = 0) -> None:
        st = dexel_offset(self.engine.ctx, self.view, self.r, self.code, self.out, self.ws, stream,
                          flags)
        if st != DEXEL_OK:
            raise DexelError(st, dexel_last_error(self.engine.ctx))

    def autotune(self, reps: int = 2, stream=None):
        """Pick the fastest kernel variant for this call (cached in the
        context for calls with the same signature)."""
        it = dexel_batch_item()
        it.in_ = self.view
        it.r = self.r
        it.op = self.code
        it.out = self.out
        return dexel_autotune(self.engine.ctx, [it], self.ws, stream, reps)

    def status(self) -> int:
        return int(self.status_t.item())

    def result(self) -> DeviceGrid:
        return DeviceGrid(self.grid.nx, self.grid.ny, self.col, self.z)


def _items(grids, radii, ops, outs):
    arr = []
    for g, r, op, o in zip(grids, radii, ops, outs):
        it = dexel_batch_item()
        it.in_ = g.view()
        it.r = float(r)
        it.op = OPS[op]
        it.out = make_out(g.nx, g.ny, o[0], o[1], o[2], o[3])
        arr.append(it)
    return arr


def batch_offset(engine: "Engine", grids, radii, ops, stream=None, max_tries: int = 8,
                 hint: int = 0):
    """Offset many shapes in one enqueue (dexel_batch_offset); returns a list
    of DeviceGrids.  Retries with a larger workspace or larger outputs."""
    grids = list(grids)
    radii = [float(r) for r in radii]
    ops = list(ops)
    dev = engine.device
    caps = [g.nseg + g.nx * g.ny + 1024 for g in grids]
    ws = outs = None
    for _ in range(max_tries):
        ws = outs = None  # the last try's buffers go before the next are made
        outs = [(torch.empty(g.nx * g.ny + 1, dtype=torch.int64, device=dev),
                 torch.empty(2 * max(c, 1), dtype=torch.float32, device=dev),
                 torch.zeros(1, dtype=torch.int64, device=dev),
                 torch.zeros(1, dtype=torch.int32, device=dev)) for g, c in zip(grids, caps)]
        items = _items(grids, radii, ops, outs)
        nbytes = dexel_batch_workspace_size(engine.ctx, items, hint)
        ws = engine.workspace(nbytes)
        st = dexel_batch_offset(engine.ctx, items, ws, stream, DEXEL_FLAG_SYNC)
        if st == DEXEL_OK:
            engine._note_hint(ws, sum(g.nseg + 2 * g.nx * g.ny for g in grids) + 1024)
            return [DeviceGrid(g.nx, g.ny, o[0], o[1]) for g, o in zip(grids, outs)]
        if st == DEXEL_ERR_WORKSPACE:
            need = dexel_workspace_need(engine.ctx, ws)
            if need <= 0:
                raise DexelError(st, dexel_last_error(engine.ctx))
            base = hint if hint > 0 else sum(g.nseg + 2 * g.nx * g.ny for g in grids) + 1024
            hint = max(int(need * 1.25) + 1024, base + base // 2)
            continue
        if st == DEXEL_ERR_CAPACITY:
            for i, o in enumerate(outs):
                if int(o[3].item()) == DEXEL_ERR_CAPACITY:
                    caps[i] = int(o[2].item()) + 1
            continue
        raise DexelError(st, dexel_last_error(engine.ctx))
    raise DexelError(DEXEL_ERR_WORKSPACE, "retries exhausted")


class BatchPlan:
    """A pre-sized batch for repeated asynchronous enqueues (and graph
    capture): construction runs the batch once synchronously to size the
    outputs and the workspace, which the plan then owns for its lifetime."""

    def __init__(self, engine: "Engine", grids, radii, ops):
        self.engine = engine
        self.grids = list(grids)
        self.radii = [float(r) for r in radii]
        self.ops = list(ops)
        res = batch_offset(engine, self.grids, self.radii, self.ops)
        dev = engine.device
        self.nseg_out = [g.nseg for g in res]
        self.nseg_in = [g.nseg for g in self.grids]
        self.outs = [(torch.empty(g.nx * g.ny + 1, dtype=torch.int64, device=dev),
                      torch.empty(2 * max(n, 1), dtype=torch.float32, device=dev),
                      torch.zeros(1, dtype=torch.int64, device=dev),
                      torch.zeros(1, dtype=torch.int32, device=dev))
                     for g, n in zip(self.grids, self.nseg_out)]
        self.items = _items(self.grids, self.radii, self.ops, self.outs)
        self.ws_bytes = dexel_batch_workspace_size(engine.ctx, self.items, engine.last_hint)
        self.ws = torch.empty(int(self.ws_bytes), dtype=torch.uint8, device=dev)

    def enqueue(self, stream=None, flags: int = 0) -> None:
        st = dexel_batch_offset(self.engine.ctx, self.items, self.ws, stream, flags)
        if st != DEXEL_OK:
            raise DexelError(st, dexel_last_error(self.engine.ctx))

    def autotune(self, reps: int = 2, stream=None):
        return dexel_autotune(self.engine.ctx, self.items, self.ws, stream, reps)

    def statuses(self):
        return [int(o[3].item()) for o in self.outs]

    def results(self):
        return [DeviceGrid(g.nx, g.ny, o[0], o[1]) for g, o in zip(self.grids, self.outs)]


_default_engine = None


def default_engine() -> Engine:
    global _default_engine
    if _default_engine is None:
        _default_engine = Engine(torch.cuda.current_device())
    return _default_engine


def offset(grid: DeviceGrid, r: float, op: str = "dilate", **kw) -> DeviceGrid:
    return default_engine().offset(grid, r, op, **kw)
