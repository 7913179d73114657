"""GPU parity of the per-column CSG (dexel_csg) and the shell, through the
C ABI, against the oracle (oracle/csg.py).

The operations copy endpoints and never compute one, so the bar is bit-exact:
column pointers and every endpoint equal to the oracle's.  The shell is the
library's dilation and erosion followed by dexel_csg; it is compared with the
oracle's shell built from the oracle's float32-model dilation and erosion,
which the offset kernels match bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import csg as ocsg
from synth import gen
from tests.helpers import HostGrid, grid_from_columns, random_grid

pytestmark = pytest.mark.gpu

OPS = ("union", "intersect", "difference")


def _dx():
    import paper_1804_08968_amd as dx
    return dx


def gpu_csg(engine, ga, gb, op):
    dx = _dx()
    out = engine.csg(dx.DeviceGrid.from_host(ga), dx.DeviceGrid.from_host(gb), op)
    col, z = out.to_host()
    return col, z.astype(np.float64)


def check(engine, ga, gb, op, label=""):
    print(f"[case] csg {label} {op} nx={ga.nx} ny={ga.ny} nseg={ga.nseg}+{gb.nseg}", flush=True)
    col, z = gpu_csg(engine, ga, gb, op)
    rc, rz = ocsg.csg(ga, gb, op)
    assert np.array_equal(col, rc), "column counts differ from the oracle"
    assert np.array_equal(z, rz), "endpoints differ from the oracle"


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("op", OPS)
def test_random_grids(engine, seed, op):
    """Several 256-column tiles and a ragged tail; up to 8 intervals per column."""
    rng = np.random.default_rng(seed)
    nx, ny = 37, 29
    ga = random_grid(rng, nx, ny, 200.0, max_per_col=8, p_empty=0.2)
    gb = random_grid(rng, nx, ny, 200.0, max_per_col=8, p_empty=0.2)
    check(engine, ga, gb, op, f"random{seed}")


def test_edge_columns(engine):
    cases = [
        ([(0.0, 2.0), (3.0, 5.0)], [(1.0, 4.0)]),
        ([(0.0, 1.0)], [(1.0, 2.0)]),                       # touching
        ([(0.0, 10.0)], [(2.0, 3.0), (5.0, 6.0)]),          # containment
        ([(0.0, 1.0), (2.0, 3.0)], [(0.0, 1.0), (2.0, 3.0)]),  # identical
        ([], [(0.0, 1.0)]),
        ([(0.0, 1.0)], []),
        ([], []),
        ([(4.0, 4.0)], [(0.0, 3.0)]),                       # zero length in A
        ([(0.0, 3.0)], [(1.0, 1.0)]),                       # zero length in B
        ([(0.0, 4.0)], [(4.0, 4.0), (5.0, 6.0)]),
        ([(-2.0 ** 100, -2.0 ** 96), (2.0 ** 96, 2.0 ** 100)], [(-5.0, 5.0)]),  # huge, exact in float32
    ]
    ca = [a for a, _ in cases]
    cb = [b for _, b in cases]
    ga = grid_from_columns(len(cases), 1, ca)
    gb = grid_from_columns(len(cases), 1, cb)
    for op in OPS:
        check(engine, ga, gb, op, "edges")
        check(engine, gb, ga, op, "edges swapped")


def test_empty_grids(engine):
    g0 = grid_from_columns(3, 2, [[] for _ in range(6)])
    rng = np.random.default_rng(3)
    g1 = random_grid(rng, 3, 2, 10.0)
    for op in OPS:
        check(engine, g0, g0, op, "both empty")
        check(engine, g0, g1, op, "empty a")
        check(engine, g1, g0, op, "empty b")


def test_self(engine):
    rng = np.random.default_rng(4)
    g = random_grid(rng, 70, 3, 100.0, max_per_col=6)
    col, z = gpu_csg(engine, g, g, "difference")
    assert col[-1] == 0
    for op in ("union", "intersect"):
        col, z = gpu_csg(engine, g, g, op)
        assert np.array_equal(col, g.col_ptr) and np.array_equal(z, g.z)


def test_capacity_reports_need(engine):
    dx = _dx()
    import torch
    rng = np.random.default_rng(5)
    ga = random_grid(rng, 8, 8, 50.0, max_per_col=5, p_empty=0.0)
    gb = random_grid(rng, 8, 8, 50.0, max_per_col=5, p_empty=0.0)
    rc, _ = ocsg.csg(ga, gb, "union")
    need = int(rc[-1])
    a, b = dx.DeviceGrid.from_host(ga), dx.DeviceGrid.from_host(gb)
    ws = engine.workspace(dx.dexel_csg_workspace_size(engine.ctx, a.view()))
    col = torch.empty(65, dtype=torch.int64, device="cuda")
    z = torch.empty(2 * (need - 1), dtype=torch.float32, device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = dx.make_out(8, 8, col, z, nout, status)
    print("[case] csg capacity", flush=True)
    st = dx.dexel_csg(engine.ctx, a.view(), b.view(), dx.DEXEL_CSG_UNION, out, ws, None, dx.DEXEL_FLAG_SYNC)
    assert st == dx.DEXEL_ERR_CAPACITY
    assert int(nout.item()) == need
    assert np.array_equal(col.cpu().numpy(), rc)


def test_host_rejects_bad_arguments(engine):
    dx = _dx()
    import torch
    rng = np.random.default_rng(6)
    ga = dx.DeviceGrid.from_host(random_grid(rng, 4, 4, 10.0))
    gb = dx.DeviceGrid.from_host(random_grid(rng, 4, 5, 10.0))
    ws = engine.workspace(dx.dexel_csg_workspace_size(engine.ctx, ga.view()))
    col = torch.empty(17, dtype=torch.int64, device="cuda")
    z = torch.empty(64, dtype=torch.float32, device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = dx.make_out(4, 4, col, z, nout, status)
    f = dx.DEXEL_FLAG_SYNC
    assert dx.dexel_csg(engine.ctx, ga.view(), gb.view(), 0, out, ws, None, f) == dx.DEXEL_ERR_INVALID
    assert dx.dexel_csg(engine.ctx, ga.view(), ga.view(), 7, out, ws, None, f) == dx.DEXEL_ERR_INVALID
    assert dx.dexel_csg(engine.ctx, ga.view(), ga.view(), 0, out, ws, None,
                        f | dx.DEXEL_FLAG_VALIDATE) == dx.DEXEL_ERR_UNSUPPORTED
    assert dx.dexel_csg(engine.ctx, ga.view(), ga.view(), 0, out, ws[:256], None,
                        f) == dx.DEXEL_ERR_WORKSPACE


def shell_check(engine, g, r, cols=None, label=""):
    dx = _dx()
    print(f"[case] shell {label} nx={g.nx} ny={g.ny} nseg={g.nseg} r={r}", flush=True)
    out = engine.shell(dx.DeviceGrid.from_host(g), r)
    col, z = out.to_host()
    z = z.astype(np.float64)
    d = oracle.run(g, r, "dilate", "f32model")
    e = oracle.run(g, r, "erode", "f32model")
    if cols is None:
        rc, rz = ocsg.csg(d, e, "difference")
        assert np.array_equal(col, rc)
        assert np.array_equal(z, rz)
        return
    for c in cols:
        want = ocsg.column_op(d.column(c), e.column(c), "difference")
        got = z[2 * col[c]: 2 * col[c + 1]].reshape(-1, 2)
        assert [tuple(v) for v in got.tolist()] == [tuple(map(float, v)) for v in want], c


@pytest.mark.parametrize("seed", [0, 1])
def test_shell_spheres(engine, oracle_lib, seed):
    g = gen.spheres_grid(seed)
    shell_check(engine, g, 3.0, label=f"c1 seed {seed}")


def test_shell_soup_crop(engine, oracle_lib):
    g = gen.config_grid("c2", 0)
    cols = []
    nx = 96
    for y in range(96):
        row = g.col_ptr[y * g.nx: y * g.nx + nx + 1]
        cols += [g.z[2 * row[x]: 2 * row[x + 1]].reshape(-1, 2).tolist() for x in range(nx)]
    crop = grid_from_columns(nx, 96, [[tuple(iv) for iv in c] for c in cols])
    shell_check(engine, crop, 4.0, label="c2 crop r=4")


def test_shell_soup_full_sampled(engine, oracle_lib):
    """The 512^2 soup at r = 4 (the scale of the paper's shell figure),
    checked on sampled columns, grid corners and borders included."""
    g = gen.config_grid("c2", 0)
    rng = np.random.default_rng(12)
    n = g.nx * g.ny
    cols = np.unique(np.concatenate([rng.integers(0, n, 600), np.arange(0, 32), np.arange(n - 32, n),
                                     np.arange(0, n, g.nx)[:32]]))
    shell_check(engine, g, 4.0, cols=cols, label="c2 full r=4")
