"""Batched offsets: many shapes of different sizes, radii and operations in
one enqueue.  Each shape's result inside the batch must equal its result
alone, bit for bit, and the oracle's float32 model, and lie within
tolerance of its float64 result."""
from __future__ import annotations

import numpy as np
import pytest

from synth import gen
from tests.helpers import compare_columns, random_grid

pytestmark = pytest.mark.gpu


def _host(dg):
    cp, z = dg.to_host()
    return cp, z.astype(np.float64)


def test_batch_equals_alone_and_oracle(engine, oracle_lib):
    import paper_1804_08968_amd as dx
    rng = np.random.default_rng(4)
    ops = ["dilate", "erode", "close", "open"]
    grids, radii, opl = [], [], []
    for i in range(14):
        nx, ny = int(rng.integers(1, 90)), int(rng.integers(1, 70))
        grids.append(random_grid(rng, nx, ny, 60.0, max_per_col=4, p_empty=0.3))
        radii.append(float(rng.uniform(0.0, 7.5)))
        opl.append(ops[i % 4])
    grids.append(gen.spheres_grid(3, n=48, count=6))
    radii.append(3.0)
    opl.append("close")
    dgs = [dx.DeviceGrid.from_host(g) for g in grids]
    print(f"[case] batch of {len(dgs)} shapes", flush=True)
    outs = dx.batch_offset(engine, dgs, radii, opl)
    for g, dg, r, op, out in zip(grids, dgs, radii, opl, outs):
        cp_b, z_b = _host(out)
        cp_a, z_a = _host(engine.offset(dg, r, op))
        assert np.array_equal(cp_b, cp_a) and np.array_equal(z_b, z_a), (g.nx, g.ny, r, op)
        ref = oracle_lib.run(g, r, op, "f32model")
        assert np.array_equal(cp_b, ref.col_ptr) and np.array_equal(z_b, ref.z), (g.nx, g.ny, r, op)
        ref64 = oracle_lib.run(g, r, op, "f64")
        res = compare_columns(np.diff(ref64.col_ptr), ref64.z, np.diff(cp_b), z_b, r,
                              k=2 if op in ("open", "close") else 1)
        assert res["failed"] == 0, (g.nx, g.ny, r, op, res)


def test_batch_c4_subset(engine, oracle_lib):
    """A few shapes of the batched workload (128^2..1024^2 primitive soups,
    radius U[2, 32]) against the oracle on sampled columns."""
    import paper_1804_08968_amd as dx
    shapes = gen.batch_shapes(0, count=6, smin=128, smax=384)
    dgs = [dx.DeviceGrid.from_host(g) for g, _ in shapes]
    radii = [r for _, r in shapes]
    ops = ["dilate", "erode", "close", "dilate", "open", "erode"]
    print("[case] c4 subset", [(g.nx, round(r, 2)) for g, r in shapes], flush=True)
    outs = dx.batch_offset(engine, dgs, radii, ops)
    rng = np.random.default_rng(1)
    for (g, r), op, out in zip(shapes, ops, outs):
        cp, z = _host(out)
        cols = np.unique(rng.integers(0, g.nx * g.ny, 200))
        if op in ("dilate", "erode"):
            c32, z32 = oracle_lib.offset_columns(g, r, op, "f32model", cols=cols)
            c64, z64 = oracle_lib.offset_columns(g, r, op, "f64", cols=cols)
        else:
            c32, z32 = oracle_lib.region_chain(g, r, op, cols, "f32model")
            c64, z64 = oracle_lib.region_chain(g, r, op, cols, "f64")
        gc = np.diff(cp)[cols]
        gz = np.concatenate([z[2 * cp[c]: 2 * cp[c + 1]] for c in cols])
        assert np.array_equal(gc, c32) and np.array_equal(gz, z32), (g.nx, r, op)
        res = compare_columns(c64, z64, gc, gz, r, k=2 if op in ("open", "close") else 1)
        assert res["failed"] == 0, res
