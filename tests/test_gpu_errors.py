"""Error handling of the C ABI on the GPU.

Every condition is forced from the host: bad arguments (rejected before any
launch), inputs the validation kernel rejects (every later kernel of the
call then exits at its first instruction), and outputs or workspaces that are
too small (the kernels' own bounds checks turn them into a status and a size
hint).  Each call that reaches the device ends normally.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import pytest

from synth import gen
from tests.helpers import HostGrid, grid_from_columns

pytestmark = pytest.mark.gpu


def _dx():
    import paper_1804_08968_amd as dx
    return dx


def _lib():
    from paper_1804_08968_amd import binding
    return binding.lib


def _out(grid, cap, nx=None, ny=None):
    import torch
    dx = _dx()
    nx = grid.nx if nx is None else nx
    ny = grid.ny if ny is None else ny
    col = torch.empty(nx * ny + 1, dtype=torch.int64, device="cuda")
    z = torch.empty(2 * max(cap, 1), dtype=torch.float32, device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    return dx.make_out(nx, ny, col, z, nout, st), (col, z, nout, st)


def _ws(engine, grid, r, op, hint=0):
    dx = _dx()
    nbytes = dx.dexel_workspace_size(engine.ctx, grid.view(), r, dx.OPS[op], hint)
    return engine.workspace(nbytes)


def _small_grid():
    g = gen.config_grid("c1", 0)
    return HostGrid(g.nx, g.ny, g.col_ptr, g.z)


def test_host_rejects_bad_arguments(engine):
    dx = _dx()
    dg = dx.DeviceGrid.from_host(_small_grid())
    ws = _ws(engine, dg, 2.0, "dilate")
    out, _ = _out(dg, dg.nseg + dg.nx * dg.ny)
    view = dg.view()
    sync = dx.DEXEL_FLAG_SYNC
    print("[case] host argument checks", flush=True)
    for r in (-1.0, float("nan"), float("inf")):
        assert dx.dexel_offset(engine.ctx, view, r, 0, out, ws, None, sync) == dx.DEXEL_ERR_INVALID
    assert dx.dexel_offset(engine.ctx, view, 300.0, 0, out, ws, None, sync) == dx.DEXEL_ERR_UNSUPPORTED
    assert dx.dexel_offset(engine.ctx, view, 2.0, 7, out, ws, None, sync) == dx.DEXEL_ERR_INVALID
    bad_out, _ = _out(dg, 16, nx=dg.nx + 1)
    assert dx.dexel_offset(engine.ctx, view, 2.0, 0, bad_out, ws, None, sync) == dx.DEXEL_ERR_INVALID
    assert "differs" in dx.dexel_last_error(engine.ctx)
    # misaligned pairs
    mis = dx.dexel_grid_view(view.nx, view.ny, view.nseg, view.col_ptr, ctypes.c_void_p(view.z + 4))
    assert dx.dexel_offset(engine.ctx, mis, 2.0, 0, out, ws, None, sync) == dx.DEXEL_ERR_INVALID
    # workspace not 256-byte aligned, and one below the minimum layout
    import torch
    st = _lib().dexel_offset(engine.ctx, ctypes.byref(view), 2.0, 0, ctypes.byref(out),
                             ctypes.c_void_p(ws.data_ptr() + 8), ws.numel() - 8,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), sync)
    assert st == dx.DEXEL_ERR_INVALID
    st = _lib().dexel_offset(engine.ctx, ctypes.byref(view), 2.0, 0, ctypes.byref(out),
                             ctypes.c_void_p(ws.data_ptr()), 512,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), sync)
    assert st == dx.DEXEL_ERR_WORKSPACE
    # a grid too large for 32-bit column ids
    big = dx.dexel_grid_view(1 << 16, 1 << 15, 0, view.col_ptr, view.z)
    nbytes = ctypes.c_size_t()
    assert _lib().dexel_workspace_size(engine.ctx, ctypes.byref(big), 2.0, 0, 0,
                                       ctypes.byref(nbytes)) == dx.DEXEL_ERR_UNSUPPORTED


def _device_status(engine, hg, r, op, flags, cap=None, nseg=None):
    dx = _dx()
    nseg = hg.nseg if nseg is None else nseg
    dg = dx.DeviceGrid.from_host(hg)
    ws = engine.workspace(dx.dexel_workspace_size(engine.ctx, dg.view(nseg), r, dx.OPS[op], 0))
    out, bufs = _out(dg, cap if cap is not None else nseg + hg.nx * hg.ny + 1024)
    st = dx.dexel_offset(engine.ctx, dg.view(nseg), r, dx.OPS[op], out, ws, None, flags)
    return st, bufs


@pytest.mark.parametrize("op", ["dilate", "erode", "close"])
@pytest.mark.parametrize("kind", ["overlap", "touching", "reversed", "nan", "inf"])
def test_validate_rejects_non_canonical(engine, kind, op):
    dx = _dx()
    cols = [[] for _ in range(12)]
    cols[3] = [(0.0, 1.0), (2.0, 3.0)]
    cols[7] = [(5.0, 6.0)]
    if kind == "overlap":
        cols[3] = [(0.0, 2.5), (2.0, 3.0)]
    elif kind == "touching":
        cols[3] = [(0.0, 2.0), (2.0, 3.0)]
    elif kind == "reversed":
        cols[7] = [(6.0, 5.0)]
    elif kind == "nan":
        cols[7] = [(float("nan"), 6.0)]
    elif kind == "inf":
        cols[7] = [(5.0, math.inf)]
    hg = grid_from_columns(4, 3, cols)
    print(f"[case] validate {kind} {op}", flush=True)
    st, bufs = _device_status(engine, hg, 1.5, op, dx.DEXEL_FLAG_SYNC | dx.DEXEL_FLAG_VALIDATE)
    assert st == dx.DEXEL_ERR_NOT_CANONICAL
    assert int(bufs[3].item()) == dx.DEXEL_ERR_NOT_CANONICAL
    assert int(bufs[2].item()) == -1


def test_validate_accepts_canonical(engine, oracle_lib):
    dx = _dx()
    hg = _small_grid()
    print("[case] validate canonical c1", flush=True)
    st, bufs = _device_status(engine, hg, 3.0, "dilate", dx.DEXEL_FLAG_SYNC | dx.DEXEL_FLAG_VALIDATE)
    assert st == dx.DEXEL_OK
    ref = oracle_lib.run(hg, 3.0, "dilate", "f32model")
    assert np.array_equal(bufs[0].cpu().numpy(), ref.col_ptr)


@pytest.mark.parametrize("kind", ["decreasing", "first_nonzero", "last_mismatch"])
def test_bad_column_pointers_always_rejected(engine, kind):
    """Column pointers are checked on every call, validation flag or not."""
    dx = _dx()
    hg = _small_grid()
    cp = hg.col_ptr.copy()
    nz = np.nonzero(np.diff(cp))[0]
    if kind == "decreasing":
        c = int(nz[len(nz) // 2]) + 1
        cp[c] = cp[c - 1] - 1 if cp[c - 1] > 0 else cp[c + 1] + 1
    elif kind == "first_nonzero":
        cp[0] = 1
    else:
        cp[-1] = cp[-1] - 1
    bad = HostGrid(hg.nx, hg.ny, cp, hg.z)
    print(f"[case] col_ptr {kind}", flush=True)
    # the view carries the true interval count; the pointers disagree with it
    st, bufs = _device_status(engine, bad, 2.0, "dilate", dx.DEXEL_FLAG_SYNC, nseg=hg.nseg)
    assert st == dx.DEXEL_ERR_NOT_CANONICAL
    assert int(bufs[3].item()) == dx.DEXEL_ERR_NOT_CANONICAL


@pytest.mark.parametrize("op", ["dilate", "erode", "open"])
def test_output_capacity_reports_need(engine, oracle_lib, op):
    """A too-small output gives CAPACITY with the needed count; a call with
    exactly that capacity succeeds and is exact."""
    dx = _dx()
    hg = _small_grid()
    ref = oracle_lib.run(hg, 2.0, op, "f32model")
    need = int(ref.col_ptr[-1])
    assert need > 2
    print(f"[case] capacity {op} need={need}", flush=True)
    st, bufs = _device_status(engine, hg, 2.0, op, dx.DEXEL_FLAG_SYNC, cap=need - 1)
    assert st == dx.DEXEL_ERR_CAPACITY
    assert int(bufs[2].item()) == need
    st, bufs = _device_status(engine, hg, 2.0, op, dx.DEXEL_FLAG_SYNC, cap=need)
    assert st == dx.DEXEL_OK
    assert np.array_equal(bufs[0].cpu().numpy(), ref.col_ptr)
    z = bufs[1].cpu().numpy()[: 2 * need].astype(np.float64)
    assert np.array_equal(z, ref.z)


@pytest.mark.parametrize("op", ["dilate", "close"])
def test_small_workspace_reports_need(engine, oracle_lib, op):
    """A workspace sized for a tiny internal capacity gives WORKSPACE and a
    capacity hint; the hinted workspace gives the exact result."""
    dx = _dx()
    hg = HostGrid(*_as_tuple(gen.config_grid("c2", 0)))
    sub = _crop(hg, 96, 80)
    dg = dx.DeviceGrid.from_host(sub)
    ref = oracle_lib.run(sub, 4.0, op, "f32model")
    print(f"[case] workspace {op} nseg={sub.nseg}", flush=True)
    import torch
    small = dx.dexel_workspace_size(engine.ctx, dg.view(), 4.0, dx.OPS[op], 64)
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    out, bufs = _out(dg, sub.nseg + sub.nx * sub.ny + 1024)
    st = dx.dexel_offset(engine.ctx, dg.view(), 4.0, dx.OPS[op], out, ws, None, dx.DEXEL_FLAG_SYNC)
    assert st == dx.DEXEL_ERR_WORKSPACE
    need = dx.dexel_workspace_need(engine.ctx, ws)
    assert need > 64
    # a call stops at the first stage that runs out, so the hint covers the
    # stages reached so far; growing it converges in a few calls
    hint = need
    for _ in range(8):
        big = dx.dexel_workspace_size(engine.ctx, dg.view(), 4.0, dx.OPS[op], hint)
        ws2 = torch.empty(big, dtype=torch.uint8, device="cuda")
        st = dx.dexel_offset(engine.ctx, dg.view(), 4.0, dx.OPS[op], out, ws2, None,
                             dx.DEXEL_FLAG_SYNC)
        if st != dx.DEXEL_ERR_WORKSPACE:
            break
        need = dx.dexel_workspace_need(engine.ctx, ws2)
        assert need > 0
        hint = max(need, 2 * hint)
    assert st == dx.DEXEL_OK, dx.dexel_last_error(engine.ctx)
    assert np.array_equal(bufs[0].cpu().numpy(), ref.col_ptr)
    n = int(ref.col_ptr[-1])
    assert np.array_equal(bufs[1].cpu().numpy()[: 2 * n].astype(np.float64), ref.z)


def test_engine_retries_to_exact_result(engine, oracle_lib):
    """Engine.offset recovers from both conditions by itself."""
    dx = _dx()
    hg = _crop(HostGrid(*_as_tuple(gen.config_grid("c2", 1))), 64, 64)
    dg = dx.DeviceGrid.from_host(hg)
    fresh = dx.Engine(0)
    try:
        print("[case] engine retry", flush=True)
        res = fresh.offset(dg, 3.0, "dilate", out_cap=1, hint=32)
        col, z = res.to_host()
        ref = oracle_lib.run(hg, 3.0, "dilate", "f32model")
        assert np.array_equal(col, ref.col_ptr)
        assert np.array_equal(z.astype(np.float64), ref.z)
    finally:
        fresh.close()


def _points_grid(nx, ny, k, height, seed):
    """k short intervals per column at random heights: a dilation's row
    unions hold several times more intervals than the input, so the call
    needs more internal capacity than the library's default (with k = 5 the
    staged kernels evaluate it: too few items per column for the direct
    evaluation or the single-interval test)."""
    rng = np.random.default_rng(seed)
    cols = []
    for _ in range(nx * ny):
        a = np.sort(rng.choice(int(height), size=k, replace=False)).astype(np.float64)
        cols.append([(float(v), float(v) + 0.25) for v in a])
    return grid_from_columns(nx, ny, cols)


def test_need_after_success_sizes_workspace(engine, oracle_lib):
    """After a call that succeeded on a roomy workspace, dexel_workspace_need
    is the largest internal buffer it used: a workspace sized with it holds
    the call again, one sized with half of it does not."""
    import torch
    dx = _dx()
    hg = _points_grid(48, 40, 5, 1500.0, 11)
    dg = dx.DeviceGrid.from_host(hg)
    r, code = 4.0, dx.OPS["dilate"]
    ref = oracle_lib.run(hg, r, "dilate", "f32model")
    default = hg.nseg + 2 * hg.nx * hg.ny + 1024
    print(f"[case] need after success nseg={hg.nseg}", flush=True)

    def call(hint):
        nbytes = dx.dexel_workspace_size(engine.ctx, dg.view(), r, code, hint)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        out, bufs = _out(dg, int(ref.col_ptr[-1]) + 1)
        st = dx.dexel_offset(engine.ctx, dg.view(), r, code, out, ws, None, dx.DEXEL_FLAG_SYNC)
        return st, ws, bufs

    st, ws, _ = call(20 * default)
    assert st == dx.DEXEL_OK, dx.dexel_last_error(engine.ctx)
    need = dx.dexel_workspace_need(engine.ctx, ws)
    assert need > default, (need, default)
    st, _, bufs = call(need)
    assert st == dx.DEXEL_OK, dx.dexel_last_error(engine.ctx)
    assert np.array_equal(bufs[0].cpu().numpy(), ref.col_ptr)
    n = int(ref.col_ptr[-1])
    assert np.array_equal(bufs[1].cpu().numpy()[: 2 * n].astype(np.float64), ref.z)
    st, _, _ = call(need // 2)
    assert st == dx.DEXEL_ERR_WORKSPACE


def test_plan_after_larger_call(oracle_lib):
    """A Plan built after the engine ran a larger call (whose workspace the
    engine keeps) sizes its own workspace from what its call used, so
    autotuning finds a variant that fits and the plan's result is exact."""
    dx = _dx()
    fresh = dx.Engine(0)
    try:
        big = dx.DeviceGrid.from_host(HostGrid(*_as_tuple(gen.config_grid("c2", 0))))
        print("[case] plan after larger call", flush=True)
        fresh.offset(big, 8.0, "dilate")
        hg = _points_grid(48, 40, 5, 1500.0, 12)
        dg = dx.DeviceGrid.from_host(hg)
        plan = dx.Plan(fresh, dg, 4.0, "dilate")
        assert fresh.last_hint > hg.nseg + 2 * hg.nx * hg.ny + 1024
        plan.autotune(reps=1)
        plan.enqueue(flags=dx.DEXEL_FLAG_SYNC)
        assert plan.status() == dx.DEXEL_OK
        col, z = plan.result().to_host()
        ref = oracle_lib.run(hg, 4.0, "dilate", "f32model")
        assert np.array_equal(col, ref.col_ptr)
        assert np.array_equal(z[: 2 * col[-1]].astype(np.float64), ref.z)
    finally:
        fresh.close()


def _as_tuple(g):
    return g.nx, g.ny, g.col_ptr, g.z


def _crop(hg, nx, ny):
    cols, lo_hi = [], []
    for y in range(ny):
        for x in range(nx):
            c = y * hg.nx + x
            a, b = hg.col_ptr[c], hg.col_ptr[c + 1]
            cols.append([(float(hg.z[2 * i]), float(hg.z[2 * i + 1])) for i in range(a, b)])
    return grid_from_columns(nx, ny, cols)
