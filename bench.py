#!/usr/bin/env python3
"""Throughput benchmark of exact dexel offsets on one MI355X.

Default workload: closing (dilation then erosion, r = 16) of a 2048 x 2048
gyroid lattice (period 64, walls about 3 voxels thick, height 2048; about 51
intervals per column, 2.15e8 intervals), the 2048^2 configuration of the
method's own scalability experiments.  One step = one closing of the whole
grid, input resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload c3|c2|c1|c4|c5|shell|slices|dexelize|tridexel|canonicalize] [--no-cpu-baseline]

value   = input intervals offset per second (intervals of the input grid per
          operation, summed over the step's operations, divided by the step
          time measured between device synchronisations).
roofline: the dominant kernel's algorithmic bytes per launch divided by its
          average duration (HIP events on the library's stream inside the
          timed region), against the 8 TB/s HBM peak.
cpu_baseline: the float64 brute-force oracle on the host cores, timed on a
          bounded sample of output columns of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = [os.path.join(ROOT, "paper_1804_08968_amd", "csrc", f)
              for f in ("dexel_kernels.hip", "dexel_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c3_close_r16_hbm_traffic.txt")


def kernels_sha256():
    """SHA-256 over the kernel source and the internal header it includes."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, each counter scaled by what it reads for a plain copy of
    known size; None if there is no summary for the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals, rows = {}, {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "kernel" and len(parts) >= 4:
                rows[parts[1]] = (float(parts[2]), float(parts[3]))
            elif len(parts) == 2:
                vals[parts[0]] = parts[1]
    if vals.get("kernels_source_sha256") != kernels_sha256() or kernel not in rows:
        return None
    copy_bytes = float(vals["copy_bytes"])
    f_scale = copy_bytes / (float(vals["copy_fetch_kib"]) * 1024.0)
    w_scale = copy_bytes / (float(vals["copy_write_kib"]) * 1024.0)
    fetch_kib, write_kib = rows[kernel]
    return (fetch_kib * f_scale + write_kib * w_scale) * 1024.0

WORKLOADS = {
    "c3": dict(desc="closing r=16 of a 2048x2048 gyroid lattice (period 64, wall ~3 voxels, "
                    "height 2048)", ops=[("close", 16.0)]),
    "c2": dict(desc="dilation and erosion at r in {2, 8, 32} of a 512x512 soup of 1350 "
                    "spheres/boxes (sizes U[4,64], height 512)",
               ops=[(op, r) for r in (2.0, 8.0, 32.0) for op in ("dilate", "erode")]),
    "c1": dict(desc="dilation r=3 of a 64x64 union of 8 spheres (R in U[4,12])",
               ops=[("dilate", 3.0)]),
    "c4": dict(desc="batched dilation of 64 primitive soups (sides log-uniform 128..1024, "
                    "20..300 spheres/boxes, per-shape radius U[2,32])", ops=[]),
    "slices": dict(desc="2D offsets (disk dilation of a slice of parallel segments) r=16 of the 2048 "
                        "rows of the 2048x2048 gyroid lattice as 2048 separate 2048x1 slices, one "
                        "batched enqueue", ops=[]),
    "dexelize": dict(desc="dexelisation on the GPU of a 2048x2048 soup of 5400 balls and boxes (sizes "
                          "U[16,256], height 2048), rays through cell centres", ops=[]),
    "tridexel": dict(desc="tri-dexel dilation r=8: the 512^3 soup of 1350 balls and boxes (the c2 primitives) "
                          "dexelised on the GPU along x, y and z, and the three 512x512 grids dilated in one "
                          "batched enqueue", ops=[]),
    "canonicalize": dict(desc="canonical form of a non-canonical 2048x2048 grid: the dexelised soup of 5400 "
                              "balls and boxes with every interval split in two overlapping halves and every "
                              "column's list reversed (47M intervals in, 23.6M out)", ops=[]),
    "shell": dict(desc="shell (dilation minus erosion, then a per-column difference) r=4 of the "
                       "512x512 soup of 1350 spheres/boxes, the grid size and radius of the paper's "
                       "shell figure", ops=[]),
    "c5": dict(desc="served stream of dilate/erode/open/close requests (r U[1,24], 30% chained "
                    "on the session's previous result) over 16 seeded shapes, sides log-uniform "
                    "256..2048, half primitive soups, half gyroids; Poisson arrivals at 0.5, 0.9 "
                    "and 1.2 x the plain server's saturation rate on the same request mix",
               ops=[]),
}


def make_grid(name):
    from synth import gen
    if name == "c3":
        return gen.gyroid_grid(0)
    if name == "c2":
        return gen.primitives_grid(0)
    if name == "c1":
        return gen.spheres_grid(0)
    raise KeyError(name)


def kernel_bytes(stage, ncols, n_in, st):
    """Algorithmic bytes of one launch of a profiled kernel: every array it
    must read or write once (CSR offsets 8 B per column, counts 4 B,
    intervals 8 B, seed tags 1 B)."""
    v0, iv, seeds, res = st["row_offset"], st["neighbour"], st["seeds"], st["result"]
    inp = 8 * (ncols + 1) + 8 * n_in
    lst_v0 = 12 * ncols + 8 * v0
    lst_i = 12 * ncols + 8 * iv
    return {
        "column_gaps": inp + 4 * ncols,
        "direct": inp + 20 * ncols + 12 * ncols + 8 * res,
        "thin_erosion": inp + ncols + 12 * ncols + 8 * res,
        "chord_extremes": 20 * ncols + ncols + 12 * ncols + 8 * res,
        "row_offset": inp + 4 * ncols + lst_v0,
        "neighbour": lst_v0 + lst_i,
        "seeds": inp + lst_i + 20 * ncols + 9 * seeds,
        "y_union": lst_v0 + 20 * ncols + 9 * seeds + 12 * ncols + 8 * res,
        "compact": 4 * ncols + 8 * (ncols + 1) + 12 * ncols + 16 * res,
    }.get(stage)


_ZERO_STATS = {"row_offset": 0, "neighbour": 0, "seeds": 0, "result": 0}


def stage_roofline(dx, per_step, pass_stats, ncols):
    """Roofline of the dominant stage over a profiled run.

    The dominant stage is the costliest by its main kernel plus its replay
    kernels (which finish the same output for the columns the main kernel
    left: overflowing lists, or every column a tiled test did not settle).
    The reported kernel is whichever of the two launch groups carries at
    least 90% of the stage's time, charged with the stage's algorithmic
    bytes; if neither does, both are reported together over the stage's
    time.  ``stage_frac`` is always the stage's bytes over the stage's time.
    One launch per pass."""
    stages = dx.PROFILE_STAGES
    modelled = [s for s in stages if kernel_bytes(s, 1, 0, _ZERO_STATS) is not None]
    tot = {s: per_step[s] + per_step.get(s + "_replay", 0.0) for s in modelled}
    dom = max(modelled, key=tot.get)
    launches = max(1, len(pass_stats))
    main_ms = per_step[dom] / launches
    rep_ms = per_step.get(dom + "_replay", 0.0) / launches
    stage_ms = tot[dom] / launches
    main_k = dx.PROFILE_KERNELS[stages.index(dom)]
    rep_k = dx.PROFILE_KERNELS[stages.index(dom + "_replay")] if dom + "_replay" in stages else None
    if rep_k is not None and rep_ms >= 0.9 * stage_ms:
        kernel, kernel_ms = rep_k, rep_ms
    elif rep_k is None or main_ms >= 0.9 * stage_ms:
        kernel, kernel_ms = main_k, main_ms
    else:
        kernel, kernel_ms = f"{main_k} + {rep_k}", stage_ms
    bpl = sum(kernel_bytes(dom, ncols, n_in, st) for n_in, st in pass_stats) / launches
    achieved = bpl / (kernel_ms / 1000.0) / 1e9 if kernel_ms > 0 else 0.0
    st_ach = bpl / (stage_ms / 1000.0) / 1e9 if stage_ms > 0 else 0.0
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
            "kernel": kernel, "kernel_ms": round(kernel_ms, 4),
            "bytes_per_launch": int(bpl), "stage": dom, "stage_ms": round(stage_ms, 4),
            "stage_frac": round(st_ach / HBM_PEAK_GBS, 5)}


def pass_bytes(ncols, n_in, st):
    """(B_alg, B_min) of one pass.  B_alg: read the input, write and read
    the x-stage pieces once (8 B of interval plus a 1-byte tag each, with
    their column offsets), write the output.  B_min: input and output
    only, what a fused pass that never stores the pieces would move."""
    ptr = 8 * (ncols + 1)
    io = ptr + 8 * n_in + ptr + 8 * st["result"]
    return io + 2 * (ptr + 9 * st["seeds"]), io


def step_roofline(pass_stats, ncols, ms_per_step):
    """Whole-step fractions of the HBM peak from B_alg and B_min."""
    b_alg = sum(pass_bytes(ncols, n, st)[0] for n, st in pass_stats)
    b_min = sum(pass_bytes(ncols, n, st)[1] for n, st in pass_stats)
    t = ms_per_step / 1000.0
    return {"step_bytes_alg": int(b_alg), "step_bytes_min": int(b_min),
            "step_frac_alg": round(b_alg / t / 1e9 / HBM_PEAK_GBS, 5),
            "step_frac_min": round(b_min / t / 1e9 / HBM_PEAK_GBS, 5)}


def measure_copy_gbs(torch, mib=1024, reps=5):
    """Device-to-device bandwidth of a plain elementwise kernel (reads and
    writes `mib` MiB), median over `reps` runs timed with HIP events."""
    nb = mib << 20
    src = torch.ones(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.add(src, 1, out=dst)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.add(src, 1, out=dst)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    del src, dst
    return round(2 * nb / (float(np.median(ts)) / 1000.0) / 1e9, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pass_list(op):
    return {"dilate": ["dilate"], "erode": ["erode"], "close": ["dilate", "erode"],
            "open": ["erode", "dilate"]}[op]


def _oracle_tile_rate(grid, op, r, budget_s):
    """Input intervals per second of the float64 oracle on a square tile of
    output columns from the grid's middle, grown until it takes about a
    quarter of `budget_s` or more."""
    import oracle
    n = 4
    while True:
        x0 = max(0, grid.nx // 2 - n // 2)
        y0 = max(0, grid.ny // 2 - n // 2)
        xs = np.arange(x0, min(grid.nx, x0 + n))
        ys = np.arange(y0, min(grid.ny, y0 + n))
        cols = (ys[:, None] * grid.nx + xs[None, :]).ravel()
        t0 = time.perf_counter()
        if op in ("dilate", "erode"):
            oracle.offset_columns(grid, r, op, "f64", cols=cols)
        else:
            oracle.region_chain(grid, r, op, cols, "f64")
        dt = time.perf_counter() - t0
        if dt * 4 > budget_s or cols.size >= grid.nx * grid.ny:
            break
        n *= 2
    per_col = grid.nseg / float(grid.nx * grid.ny)
    segs = cols.size * per_col
    return segs / dt, (f"{n}x{n} tile of output columns ({cols.size} columns, {segs:.0f} "
                       f"input-interval equivalents at {per_col:.2f} per column), {dt:.2f} s")


def cpu_baseline(grid, ops, budget_s=20.0):
    """Time the float64 oracle on a tile of output columns, on every host
    thread it uses and on one thread."""
    import oracle
    op, r = ops[0]
    cores = oracle.num_threads()
    v_all, s_all = _oracle_tile_rate(grid, op, r, budget_s)
    oracle.set_num_threads(1)
    try:
        v_one, s_one = _oracle_tile_rate(grid, op, r, budget_s / 2)
    finally:
        oracle.set_num_threads(cores)
    return {"value": v_all, "unit": "input segments/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{op} r={r} on a {s_all}",
            "one_thread": {"value": v_one, "sample": f"{op} r={r} on a {s_one}"}}


def csg_bytes(ncols, na, nb, nout):
    """Algorithmic bytes of one dexel_csg: both inputs read once, the output
    written once (CSR offsets 8 B per column, intervals 8 B), per-column
    counts written and read (4 B each) and the scan written and read (8 B)."""
    return 3 * 8 * (ncols + 1) + 8 * (na + nb + nout) + 2 * 4 * ncols + 2 * 8 * (ncols + 1)


def run_tridexel(args, dx, torch):
    """tridexel: dexelisation along the three axes and the dilation of each
    direction, all on the device, the primitive records resident in HBM."""
    import oracle
    from synth import gen
    n, r = 512, 8.0
    rec = gen.primitive_records(0)           # the c2 soup's primitives
    eng = dx.Engine(0)
    prims = torch.as_tensor(rec, dtype=torch.float64).cuda().contiguous()
    axes = ("x", "y", "z")
    tri = eng.tridexel((n, n, n), prims)     # sizes the grids
    calls = []
    for a in axes:
        g = tri[a]
        nout = torch.zeros(1, dtype=torch.int64, device="cuda")
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = torch.empty(dx.dexel_dexelize_workspace_size(eng.ctx, g.nx, g.ny), dtype=torch.uint8, device="cuda")
        calls.append((g, dx.make_out(g.nx, g.ny, g.col_ptr, g.z, nout, status), ws, dx.RAY_FLAGS[a], status))
    nseg = {a: tri[a].nseg for a in axes}
    n_in = sum(nseg.values())
    ncols = sum(tri[a].nx * tri[a].ny for a in axes)
    bp = dx.BatchPlan(eng, [tri[a] for a in axes], [r] * 3, ["dilate"] * 3)
    chosen, var_ms = bp.autotune(reps=2)
    bp.enqueue(flags=dx.DEXEL_FLAG_SYNC)
    stats = dx.dexel_workspace_stats(eng.ctx, bp.ws)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]

    def step(i=None):
        if i is not None:
            ev[i][0].record()
        for g, out, ws, fl, _ in calls:
            st = dx.dexel_dexelize(eng.ctx, g.nx, g.ny, prims, out, ws, None, fl)
            if st != dx.DEXEL_OK:
                raise RuntimeError(f"dexel_dexelize enqueue failed: {st}")
        if i is not None:
            ev[i][1].record()
        bp.enqueue()
        if i is not None:
            ev[i][2].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dx.dexel_profile_read(eng.ctx, reset=True)
    dx.dexel_profile_enable(eng.ctx, True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    te = time.perf_counter()
    dx.dexel_profile_enable(eng.ctx, False)
    prof_ms, _ = dx.dexel_profile_read(eng.ctx, reset=True)
    bad = [int(c[4].item()) for c in calls if int(c[4].item()) != 0] + [s_ for s_ in bp.statuses() if s_ != 0]
    if bad:
        raise RuntimeError(f"device statuses {bad}")
    if any(tri[a].nseg != nseg[a] for a in axes):
        raise RuntimeError("dexelisation changed between steps")
    ms_step = (te - ts) * 1000.0 / args.steps
    dex_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    off_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    stages = dx.PROFILE_STAGES
    per_step = {s_: prof_ms[i] / args.steps for i, s_ in enumerate(stages)}
    roof = stage_roofline(dx, per_step, [(n_in, stats)], ncols)
    line = {
        "metric": "input dexel segments offset/sec",
        "value": n_in / (ms_step / 1000.0),
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"tridexel: {WORKLOADS['tridexel']['desc']}", "grid": f"{n}x{n}x{n}",
                   "primitives": len(rec), "r": r, "nseg_in": nseg},
        "dexelize_ms_per_step": round(dex_ms, 4),
        "offset_ms_per_step": round(off_ms, 4),
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "variant": chosen,
    }
    if not args.no_cpu_baseline:
        # the oracle's dilation of the z-ray grid (the generator's c2 grid) on
        # a square tile of output columns, grown until it takes a few seconds
        grid = gen.primitives_grid(0)
        t, best = 8, None
        while True:
            x0, y0 = grid.nx // 2 - t // 2, grid.ny // 2 - t // 2
            cols = (np.arange(y0, y0 + t)[:, None] * grid.nx + np.arange(x0, x0 + t)[None, :]).ravel()
            tc = time.perf_counter()
            oracle.offset_columns(grid, r, "dilate", "f64", cols=cols)
            dt = time.perf_counter() - tc
            best = (cols.size, dt, t)
            if dt * 4 > args.cpu_budget or t >= min(grid.nx, grid.ny):
                break
            t *= 2
        nc, dt, t = best
        per_col = grid.nseg / float(grid.nx * grid.ny)
        line["cpu_baseline"] = {"value": nc * per_col / dt, "unit": "input segments/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"dilation r={r} of the z-ray grid on a {t}x{t} tile of output "
                                          f"columns ({nc} columns, {nc * per_col:.0f} input-interval "
                                          f"equivalents), {dt:.2f} s; the oracle's dexelisation (pure "
                                          f"Python) is not included"}
    print(json.dumps(line), flush=True)
    eng.close()


def run_canonicalize(args, dx, torch):
    """canonicalize: dexel_canonicalize of a grid whose columns hold split,
    reversed intervals; inputs resident in HBM."""
    from oracle import canonical as oc
    from synth import gen
    n, count = 2048, 5400
    rec = gen.primitive_records(7, n=n, count=count, smin=16.0, smax=256.0, height=float(n))
    eng = dx.Engine(0)
    soup = eng.dexelize(n, n, rec)
    cp, z = soup.to_host()
    ncols = n * n
    pairs = z.reshape(-1, 2)
    mid = (np.float32(0.5) * (pairs[:, 0] + pairs[:, 1])).astype(np.float32)
    halves = np.stack([np.stack([pairs[:, 0], mid], 1), np.stack([mid, pairs[:, 1]], 1)], 1).reshape(-1, 2)
    cp2 = 2 * cp
    cnt2 = np.diff(cp2)
    col = np.repeat(np.arange(ncols), cnt2)
    j = np.arange(cp2[-1])
    src = cp2[col] + cp2[col + 1] - 1 - j          # each column's list reversed
    messy = np.ascontiguousarray(halves[src]).reshape(-1)
    del halves, col, j, src
    n_in = int(cp2[-1])
    in_ptr = torch.as_tensor(cp2, dtype=torch.int64).cuda()
    in_z = torch.as_tensor(messy, dtype=torch.float32).cuda()
    view = dx.make_view(n, n, in_ptr, in_z, n_in)
    out_ptr = torch.empty(ncols + 1, dtype=torch.int64, device="cuda")
    out_z = torch.empty(2 * n_in, dtype=torch.float32, device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = dx.make_out(n, n, out_ptr, out_z, nout, status)
    ws = torch.empty(dx.dexel_canonicalize_workspace_size(eng.ctx, view), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        dx.dexel_canonicalize(eng.ctx, view, out, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        st = dx.dexel_canonicalize(eng.ctx, view, out, ws)
        if st != dx.DEXEL_OK:
            raise RuntimeError(f"dexel_canonicalize enqueue failed: {st}")
    e1.record()
    torch.cuda.synchronize()
    te = time.perf_counter()
    if int(status.item()) != 0:
        raise RuntimeError(f"dexel_canonicalize status {int(status.item())}")
    n_out = int(nout.item())
    if n_out != int(cp[-1]) or not torch.equal(out_ptr.cpu(), torch.as_tensor(cp)):
        raise RuntimeError("canonical form differs from the dexelised soup")
    ms_step = (te - ts) * 1000.0 / args.steps
    ev_ms = e0.elapsed_time(e1) / args.steps
    nbytes = 8 * (ncols + 1) + 8 * n_in + 8 * (ncols + 1) + 8 * n_out
    gbs = nbytes / (ev_ms / 1000.0) / 1e9
    line = {
        "metric": "input dexel intervals canonicalised/sec",
        "value": n_in / (ms_step / 1000.0),
        "unit": "intervals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"canonicalize: {WORKLOADS['canonicalize']['desc']}", "grid": f"{n}x{n}",
                   "nseg_in": n_in, "nseg_out": n_out},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "k_canon, k_canon_long (count and write passes) and the scan",
                     "kernel_ms": round(ev_ms, 4), "bytes_per_launch": int(nbytes)},
    }
    if not args.no_cpu_baseline:
        # the oracle on whole grid rows from the middle until about the CPU budget
        tc, rows, done = time.perf_counter(), 0, 0
        y = n // 2
        pr = messy.reshape(-1, 2).astype(np.float64)
        while time.perf_counter() - tc < args.cpu_budget / 2 and rows < n:
            for x in range(n):
                c = (y + rows) * n + x
                oc.column(pr[cp2[c]:cp2[c + 1]])
                done += int(cp2[c + 1] - cp2[c])
            rows += 1
        dt = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": done / dt, "unit": "intervals/s", "cores": 1, "kind": "oracle",
                                "sample": f"{rows} grid rows from the middle ({rows * n} columns, {done} input "
                                          f"intervals), {dt:.2f} s, pure Python, one thread"}
    print(json.dumps(line), flush=True)
    eng.close()


def run_shell(args, dx, torch):
    """shell: dilation, erosion and the per-column difference of the 512^2
    soup at r = 4, all on the device, inputs resident in HBM."""
    import oracle
    from oracle import csg as ocsg
    r = 4.0
    t0 = time.perf_counter()
    grid = make_grid("c2")
    eng = dx.Engine(0)
    dg = dx.DeviceGrid.from_host(grid)
    ncols = grid.nx * grid.ny
    pd_, pe_ = dx.Plan(eng, dg, r, "dilate"), dx.Plan(eng, dg, r, "erode")
    variants = [pd_.autotune(reps=2)[0], pe_.autotune(reps=2)[0]]
    pass_stats = []
    for p in (pd_, pe_):
        p.enqueue(flags=dx.DEXEL_FLAG_SYNC)
        pass_stats.append((dg.nseg, dx.dexel_workspace_stats(eng.ctx, p.ws)))
    nd, ne = pd_.nseg_out, pe_.nseg_out
    va = dx.make_view(grid.nx, grid.ny, pd_.col, pd_.z, nd)
    vb = dx.make_view(grid.nx, grid.ny, pe_.col, pe_.z, ne)
    cap = nd + ne + 1
    col = torch.empty(ncols + 1, dtype=torch.int64, device="cuda")
    z = torch.empty(2 * cap, dtype=torch.float32, device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = dx.make_out(grid.nx, grid.ny, col, z, nout, status)
    ws_csg = torch.empty(dx.dexel_csg_workspace_size(eng.ctx, va), dtype=torch.uint8, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def step(i=None):
        pd_.enqueue()
        pe_.enqueue()
        if i is not None:
            ev[i][0].record()
        st = dx.dexel_csg(eng.ctx, va, vb, dx.DEXEL_CSG_DIFFERENCE, out, ws_csg, None, 0)
        if i is not None:
            ev[i][1].record()
        if st != dx.DEXEL_OK:
            raise RuntimeError(f"dexel_csg enqueue failed: {st}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dx.dexel_profile_read(eng.ctx, reset=True)
    dx.dexel_profile_enable(eng.ctx, True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    te = time.perf_counter()
    dx.dexel_profile_enable(eng.ctx, False)
    prof_ms, _ = dx.dexel_profile_read(eng.ctx, reset=True)
    for p in (pd_, pe_):
        if p.status() != 0:
            raise RuntimeError(f"device status {p.status()}")
    if int(status.item()) != 0:
        raise RuntimeError(f"dexel_csg status {int(status.item())}")
    nshell = int(nout.item())
    ms_step = (te - ts) * 1000.0 / args.steps
    csg_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    stages = dx.PROFILE_STAGES
    per_step = {s_: prof_ms[i] / args.steps for i, s_ in enumerate(stages)}
    roof = stage_roofline(dx, per_step, pass_stats, ncols)
    cb = csg_bytes(ncols, nd, ne, nshell)
    csg_gbs = cb / (csg_ms / 1000.0) / 1e9
    line = {
        "metric": "input dexel segments offset/sec",
        "value": grid.nseg / (ms_step / 1000.0),
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"shell: {WORKLOADS['shell']['desc']}", "grid": f"{grid.nx}x{grid.ny}",
                   "nseg_in": grid.nseg, "r": r, "nseg_dilation": nd, "nseg_erosion": ne,
                   "nseg_shell": nshell},
        "roofline": roof,
        "csg": {"bound": "hbm", "achieved": round(csg_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(csg_gbs / HBM_PEAK_GBS, 5), "kernels": "k_csg_count, scan, k_csg_write",
                "ms_per_call": round(csg_ms, 4), "bytes_per_call": int(cb)},
        "kernels_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "variants": variants,
    }
    if not args.no_cpu_baseline:
        # the oracle's shell on a square tile of output columns, grown until
        # it takes a few seconds
        n, best = 8, None
        while True:
            x0, y0 = grid.nx // 2 - n // 2, grid.ny // 2 - n // 2
            cols = (np.arange(y0, y0 + n)[:, None] * grid.nx + np.arange(x0, x0 + n)[None, :]).ravel()
            tc = time.perf_counter()
            cd, zd = oracle.offset_columns(grid, r, "dilate", "f64", cols=cols)
            ce, ze = oracle.offset_columns(grid, r, "erode", "f64", cols=cols)
            od, oe = np.concatenate([[0], np.cumsum(cd)]), np.concatenate([[0], np.cumsum(ce)])
            for k in range(cols.size):
                ocsg.column_op(zd[2 * od[k]: 2 * od[k + 1]], ze[2 * oe[k]: 2 * oe[k + 1]], "difference")
            dt = time.perf_counter() - tc
            best = (cols.size, dt, n)
            if dt * 4 > args.cpu_budget or n >= min(grid.nx, grid.ny):
                break
            n *= 2
        nc, dt, n = best
        per_col = grid.nseg / float(ncols)
        line["cpu_baseline"] = {"value": nc * per_col / dt, "unit": "input segments/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"shell r={r} on a {n}x{n} tile of output columns ({nc} "
                                          f"columns, {nc * per_col:.0f} input-interval equivalents), "
                                          f"{dt:.2f} s"}
    print(json.dumps(line), flush=True)
    eng.close()


def run_slices(args, dx, torch):
    """slices: the 2D method of Sec. 3.2 on many slices in one batch."""
    import oracle
    from synth import gen
    r = 16.0
    t0 = time.perf_counter()
    g = gen.gyroid_grid(0)
    nx, ny = g.nx, g.ny
    eng = dx.Engine(0)
    cp = torch.as_tensor(g.col_ptr, dtype=torch.int64).cuda()
    z = torch.as_tensor(g.z.reshape(-1), dtype=torch.float32).cuda()
    slices = []
    for y in range(ny):
        b0, b1 = int(g.col_ptr[y * nx]), int(g.col_ptr[(y + 1) * nx])
        col = (cp[y * nx:(y + 1) * nx + 1] - b0).contiguous()
        zz = z[2 * b0: 2 * b1] if b1 > b0 else torch.zeros(2, dtype=torch.float32, device="cuda")
        slices.append(dx.DeviceGrid(nx, 1, col, zz))
    bp = dx.BatchPlan(eng, slices, [r] * ny, ["dilate"] * ny)
    chosen, _ = bp.autotune(reps=2)
    print(f"[bench] slices ready ({time.perf_counter() - t0:.1f} s), variant {chosen}", file=sys.stderr,
          flush=True)
    bp.enqueue(flags=dx.DEXEL_FLAG_SYNC)
    st = dx.dexel_workspace_stats(eng.ctx, bp.ws)
    for _ in range(args.warmup):
        bp.enqueue()
    torch.cuda.synchronize()
    dx.dexel_profile_read(eng.ctx, reset=True)
    dx.dexel_profile_enable(eng.ctx, True)
    ts = time.perf_counter()
    for _ in range(args.steps):
        bp.enqueue()
    torch.cuda.synchronize()
    te = time.perf_counter()
    dx.dexel_profile_enable(eng.ctx, False)
    prof_ms, _ = dx.dexel_profile_read(eng.ctx, reset=True)
    bad = [s_ for s_ in bp.statuses() if s_ != 0]
    if bad:
        raise RuntimeError(f"device status {bad[0]}")
    ms_step = (te - ts) * 1000.0 / args.steps
    stages = dx.PROFILE_STAGES
    per_step = {s_: prof_ms[i] / args.steps for i, s_ in enumerate(stages)}
    ncols = nx * ny
    roof = stage_roofline(dx, per_step, [(g.nseg, st)], ncols)
    line = {
        "metric": "input dexel segments offset/sec",
        "value": g.nseg / (ms_step / 1000.0),
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"slices: {WORKLOADS['slices']['desc']}", "slices": ny,
                   "columns_per_slice": nx, "nseg_in": g.nseg, "r": r,
                   "nseg_out": sum(o for o in bp.nseg_out)},
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "variant": chosen,
    }
    if not args.no_cpu_baseline:
        done, segs, tc = 0, 0, time.perf_counter()
        for y in range(ny):
            b0, b1 = int(g.col_ptr[y * nx]), int(g.col_ptr[(y + 1) * nx])
            h = oracle.Grid(nx, 1, g.col_ptr[y * nx:(y + 1) * nx + 1] - b0,
                            np.asarray(g.z, dtype=np.float64).reshape(-1)[2 * b0: 2 * b1])
            oracle.offset(h, r, "dilate", "f64")
            done += 1
            segs += b1 - b0
            if time.perf_counter() - tc > args.cpu_budget / 2:
                break
        dt = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": segs / dt, "unit": "input segments/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"the first {done} slices in full ({segs} intervals), {dt:.2f} s"}
    print(json.dumps(line), flush=True)
    eng.close()


# float64 operations of one ball test (two differences, three products, a sum,
# a compare) and one box test (four differences, four roundings, four compares)
DEX_FLOPS_PER_TEST = 7
FP64_VECTOR_PEAK_TFLOPS = 78.6


def dex_candidate_pairs(rec, n):
    """(column, primitive) pairs whose column lies in the primitive's cell
    bounding box (a ball's square of side 2R, a box's cell range), clipped to
    the n x n grid: the tests an exact dexeliser with bounding-box culling
    cannot skip."""
    import numpy as np
    rec = np.asarray(rec, dtype=np.float64)
    ball = rec[:, 0] == 0.0
    lo = np.where(ball[:, None], rec[:, 1:3] - rec[:, 4:5], rec[:, 1:3])
    hi = np.where(ball[:, None], rec[:, 1:3] + rec[:, 4:5], rec[:, 4:6])
    a = np.clip(np.ceil(lo - 0.5), 0, n)
    b = np.clip(np.floor(hi - 0.5), -1, n - 1)
    w = np.maximum(b - a + 1, 0)
    return int(np.sum(w[:, 0] * w[:, 1]))


def run_dexelize(args, dx, torch):
    """dexelize: primitives to a dexel grid on the device."""
    from oracle import dexelize as od
    from synth import gen
    n, count = 2048, 5400
    kw = dict(n=n, count=count, smin=16.0, smax=256.0, height=float(n))
    rec = gen.primitive_records(7, **kw)
    eng = dx.Engine(0)
    prims = torch.as_tensor(rec, dtype=torch.float64).cuda().contiguous()
    res = eng.dexelize(n, n, prims)          # sizes the output
    nseg = res.nseg
    ncols = n * n
    col = torch.empty(ncols + 1, dtype=torch.int64, device="cuda")
    z = torch.empty(2 * max(nseg, 1), dtype=torch.float32, device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = dx.make_out(n, n, col, z, nout, status)
    ws = torch.empty(dx.dexel_dexelize_workspace_size(eng.ctx, n, n), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        dx.dexel_dexelize(eng.ctx, n, n, prims, out, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        st = dx.dexel_dexelize(eng.ctx, n, n, prims, out, ws)
        if st != dx.DEXEL_OK:
            raise RuntimeError(f"dexel_dexelize enqueue failed: {st}")
    e1.record()
    torch.cuda.synchronize()
    te = time.perf_counter()
    if int(status.item()) != 0:
        raise RuntimeError(f"dexel_dexelize status {int(status.item())}")
    ms_step = (te - ts) * 1000.0 / args.steps
    ev_ms = e0.elapsed_time(e1) / args.steps
    pairs = dex_candidate_pairs(rec, n)
    tflops = pairs * DEX_FLOPS_PER_TEST / (ev_ms / 1000.0) / 1e12
    line = {
        "metric": "dexel intervals produced/sec",
        "value": nseg / (ms_step / 1000.0),
        "unit": "intervals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dexelize: {WORKLOADS['dexelize']['desc']}", "grid": f"{n}x{n}",
                   "primitives": count, "nseg_out": nseg},
        "roofline": {"bound": "alu", "achieved": round(tflops, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 5),
                     "traffic": None, "kernel": "k_dexelize (count and write passes)",
                     "kernel_ms": round(ev_ms, 4),
                     "candidate_pairs": pairs, "flops_per_launch": int(pairs * DEX_FLOPS_PER_TEST)},
    }
    if not args.no_cpu_baseline:
        # the oracle on whole grid rows until about half the CPU budget
        prims_l = [tuple(p) for p in rec]
        tc, rows, made = time.perf_counter(), 0, 0
        y = n // 2
        while time.perf_counter() - tc < args.cpu_budget / 2 and rows < n:
            for x in range(n):
                made += len(od.merge(od.column_intervals(x, y + rows, prims_l)))
            rows += 1
        dt = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": made / dt, "unit": "intervals/s", "cores": 1, "kind": "oracle",
                                "sample": f"{rows} grid rows from the middle ({rows * n} columns, {made} "
                                          f"intervals), {dt:.2f} s, pure Python, one thread"}
    print(json.dumps(line), flush=True)
    eng.close()


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def run_batch(args, dx, torch):
    """c4: one batched enqueue (autotuned kernel variant, replayed from a
    captured HIP graph) against 64 plain per-shape calls on the same stream."""
    from synth import gen
    t0 = time.perf_counter()
    shapes = gen.batch_shapes(0)
    grids = [g for g, _ in shapes]
    radii = [r for _, r in shapes]
    ops = ["dilate"] * len(grids)
    n_in = sum(g.nseg for g in grids)
    print(f"[bench] c4: {len(grids)} shapes, {n_in} intervals, "
          f"{sum(g.nx * g.ny for g in grids)} columns ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    eng = dx.Engine(0)
    dgs = [dx.DeviceGrid.from_host(g) for g in grids]

    # plain: one call per shape, completion time of each shape from the step start
    plans = [dx.Plan(eng, dg, r, op) for dg, r, op in zip(dgs, radii, ops)]
    for _ in range(args.warmup):
        for p in plans:
            p.enqueue()
    torch.cuda.synchronize()
    plain_ms, lat_plain = [], []
    for _ in range(args.steps):
        ev0 = torch.cuda.Event(enable_timing=True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in plans]
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        ev0.record()
        for p, e in zip(plans, evs):
            p.enqueue()
            e.record()
        torch.cuda.synchronize()
        plain_ms.append((time.perf_counter() - t_a) * 1000.0)
        lat_plain.extend(ev0.elapsed_time(e) for e in evs)

    # batched: autotune the kernel variant, capture the enqueue in a graph
    bp = dx.BatchPlan(eng, dgs, radii, ops)
    chosen, var_ms = bp.autotune(reps=2)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cap_stream = torch.cuda.Stream()
    cap_stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap_stream):
        bp.enqueue()  # warm on the capture stream
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=cap_stream):
        bp.enqueue(stream=cap_stream)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    batch_ms = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        batch_ms.append((time.perf_counter() - t_a) * 1000.0)
    if any(st != 0 for st in bp.statuses()):
        raise RuntimeError(f"batch statuses {bp.statuses()}")

    # kernel breakdown of one eager batched enqueue (profiled, outside the graph)
    dx.dexel_profile_read(eng.ctx, reset=True)
    dx.dexel_profile_enable(eng.ctx, True)
    bp.enqueue()
    torch.cuda.synchronize()
    dx.dexel_profile_enable(eng.ctx, False)
    prof_ms, passes = dx.dexel_profile_read(eng.ctx, reset=True)
    per = {s: prof_ms[i] for i, s in enumerate(dx.PROFILE_STAGES)}
    dom = max(per, key=per.get)
    # the batch is one pass over every shape's columns: its list sizes are
    # the workspace header's totals, its launches one per stage
    ncols_b = sum(g.nx * g.ny for g in grids)
    roof = stage_roofline(dx, per, [(n_in, dx.dexel_workspace_stats(eng.ctx, bp.ws))], ncols_b)

    ms_step = float(np.median(batch_ms))
    value = n_in / (ms_step / 1000.0)
    line = {
        "metric": "input dexel segments offset/sec",
        "value": value,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"c4: {WORKLOADS['c4']['desc']}", "shapes": len(grids),
                   "nseg_in": n_in, "ops": "dilate"},
        "batched": {"ms_per_step": ms_step, "latency_ms_p50": ms_step, "latency_ms_p99": ms_step,
                    "variant": chosen, "variant_ms": [round(v, 3) for v in var_ms],
                    "graph": True},
        "plain": {"ms_per_step": float(np.median(plain_ms)),
                  "segments_per_s": n_in / (float(np.median(plain_ms)) / 1000.0),
                  "latency_ms_p50": pct(lat_plain, 50), "latency_ms_p99": pct(lat_plain, 99)},
        "speedup_vs_plain": float(np.median(plain_ms)) / ms_step,
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v, 4) for k, v in per.items()},
        "dominant_kernel": dx.PROFILE_KERNELS[dx.PROFILE_STAGES.index(dom)],
    }
    if not args.no_cpu_baseline:
        import oracle
        t_c = time.perf_counter()
        done_seg, done = 0, 0
        for g0, r0 in zip(grids, radii):
            oracle.offset_columns(g0, r0, "dilate", "f64")
            done_seg += g0.nseg
            done += 1
            if time.perf_counter() - t_c > args.cpu_budget:
                break
        dt = time.perf_counter() - t_c
        line["cpu_baseline"] = {"value": done_seg / dt, "unit": "input segments/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"full dilation of the first {done} batch shapes in "
                                          f"order ({done_seg} intervals), {dt:.2f} s"}
    print(json.dumps(line), flush=True)
    eng.close()


def run_serving(args, dx, torch):
    """c5: continuous batching against a plain one-request-at-a-time server."""
    from paper_1804_08968_amd import serve
    from synth import gen
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    eng = dx.Engine(0)
    pool = []
    for i in range(16):
        side = int(round(np.exp(rng.uniform(np.log(256), np.log(2048)))))
        sub = int(rng.integers(0, 2**31 - 1))
        if i % 2 == 0:
            # soups are dexelised on the device from their primitive records
            rec = gen.primitive_records(sub, n=side, count=int(rng.integers(20, 301)),
                                        smin=4.0 * side / 512, smax=64.0 * side / 512, height=float(side))
            pool.append(eng.dexelize(side, side, rec))
        else:
            pool.append(dx.DeviceGrid.from_host(gen.gyroid_grid(sub, n=side)))
    print(f"[bench] c5 pool: sides {[g.nx for g in pool]}, "
          f"{sum(g.nseg for g in pool)} intervals ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    ops = ["dilate", "erode", "open", "close"]

    def make(n, rate, seed):
        r1 = np.random.default_rng(seed)
        r2 = np.random.default_rng(seed + 7)
        t, out = 0.0, []
        for i in range(n):
            t += 0.0 if rate is None else r2.exponential(1.0 / rate)
            out.append(serve.Request(i, t, int(r1.integers(0, len(pool))),
                                     ops[int(r1.integers(0, 4))], float(r1.uniform(1.0, 24.0)),
                                     bool(r1.random() < 0.3), int(r1.integers(0, 16))))
        return out

    # warm the library (LUTs, kernel code) and measure the plain service rate
    serve.Server(eng, pool, mode="plain", keep_results=False).run(make(4, None, 99))
    sat_reqs = make(args.serve_requests, None, 2)  # the same mix as the loaded runs
    sat_done = serve.Server(eng, pool, mode="plain", keep_results=False).run(sat_reqs)
    sat = serve.summarize(sat_done)
    print(f"[bench] saturation run {sat}", file=sys.stderr, flush=True)
    # service time of each request of the plain run (one request on the GPU at
    # a time, back to back): which requests take the time
    kinds = ["soup" if i % 2 == 0 else "gyroid" for i in range(len(pool))]
    prev, svc = 0.0, []
    by_id = {q.id: q for q in sat_reqs}
    for d in sorted(sat_done, key=lambda d: d.done):
        q = by_id[d.id]
        begin = max(prev, d.start)
        g = pool[q.shape]
        svc.append({"id": q.id, "op": q.op, "r": round(q.r, 2), "chain": q.chain,
                    "shape": f"{kinds[q.shape]} {g.nx}^2", "nseg_in": d.nseg_in,
                    "service_ms": round((d.done - begin) * 1000.0, 2)})
        prev = d.done
    slowest = sorted(svc, key=lambda v: -v["service_ms"])[:8]
    for v in slowest:
        print(f"[bench] slow plain request {v}", file=sys.stderr, flush=True)
    if not sat["completed"] or not sat["makespan_s"]:
        raise RuntimeError(f"saturation run completed nothing: {sat}")
    mu = sat["completed"] / sat["makespan_s"]
    print(f"[bench] plain saturation rate {mu:.2f} req/s", file=sys.stderr, flush=True)
    table = []
    for f in (0.5, 0.9, 1.2):
        reqs = make(args.serve_requests, f * mu, 2)
        row = {"load": f, "rate_req_s": f * mu}
        for mode in ("continuous", "plain"):
            srv = serve.Server(eng, pool, mode=mode, max_batch=16, slots=2, keep_results=False,
                               policy=args.serve_policy)
            row[mode] = serve.summarize(srv.run(reqs))
            print(f"[bench] load {f}: {mode} {row[mode]}", file=sys.stderr, flush=True)
        table.append(row)
    top = table[-1]["continuous"]
    line = {
        "metric": "input dexel segments offset/sec",
        "value": top["segments_per_s"],
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.serve_requests,
        "warmup": 4,
        "ms_per_step": top["makespan_s"] * 1000.0 / max(1, top["completed"]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"c5: {WORKLOADS['c5']['desc']}",
                   "requests_per_load": args.serve_requests, "max_batch": 16, "slots": 2,
                   "policy": args.serve_policy,
                   "budget_bytes": 64 << 30},
        "serving": {"saturation_req_s_plain": mu, "loads": table, "slowest_plain": slowest,
                    "service_ms_total_plain": round(sum(v["service_ms"] for v in svc), 1)},
        "latency_ms_p50": top["latency_ms_p50"],
        "latency_ms_p99": top["latency_ms_p99"],
    }
    print(json.dumps(line), flush=True)
    eng.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--serve-requests", type=int, default=60)
    ap.add_argument("--serve-policy", default="fifo", choices=["fifo", "sjf"],
                    help="c5 continuous server's admission order")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one elementwise kernel over this many MiB (reads and writes "
                         "a known number of bytes: the reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the offset of one "
              "grid is not split across GPUs by this library.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1804_08968_amd as dx

    if args.calibrate_copy > 0:
        # an elementwise kernel that reads nb bytes and writes nb bytes
        # (a device-to-device copy_ may go to a DMA engine, not a kernel)
        nb = args.calibrate_copy << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] calibration kernel: {nb} bytes read, {nb} bytes written", file=sys.stderr,
              flush=True)
        del src, dst

    if args.workload == "c4":
        return run_batch(args, dx, torch)
    if args.workload == "c5":
        return run_serving(args, dx, torch)
    if args.workload == "shell":
        return run_shell(args, dx, torch)
    if args.workload == "slices":
        return run_slices(args, dx, torch)
    if args.workload == "dexelize":
        return run_dexelize(args, dx, torch)
    if args.workload == "tridexel":
        return run_tridexel(args, dx, torch)
    if args.workload == "canonicalize":
        return run_canonicalize(args, dx, torch)
    wl = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    grid = make_grid(args.workload)
    print(f"[bench] workload {args.workload}: {grid.nx}x{grid.ny}, {grid.nseg} intervals "
          f"(generated in {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    eng = dx.Engine(0)
    dg = dx.DeviceGrid.from_host(grid)
    ncols = grid.nx * grid.ny

    # per-pass sizes for the algorithmic-byte model (outside the timed region)
    pass_stats = []
    for op, r in wl["ops"]:
        cur = dg
        for p in pass_list(op):
            plan = dx.Plan(eng, cur, r, p)
            plan.enqueue(flags=dx.DEXEL_FLAG_SYNC)
            st = dx.dexel_workspace_stats(eng.ctx, plan.ws)
            pass_stats.append((cur.nseg, st))
            cur = plan.result()
    plans = [dx.Plan(eng, dg, r, op) for op, r in wl["ops"]]
    variants = [p.autotune(reps=2)[0] for p in plans]
    print(f"[bench] plans ready, variants {variants} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        for p in plans:
            p.enqueue()
    torch.cuda.synchronize()

    # timed region: K whole steps with the library's profiling events off;
    # one HIP event per step boundary on the stream the plans run on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        for p in plans:
            p.enqueue()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    for p in plans:
        if p.status() != 0:
            raise RuntimeError(f"device status {p.status()} for {p.op}")
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]

    # kernel breakdown: the same K steps again with the library's stage
    # events on (recorded on its stream), for the roofline
    dx.dexel_profile_read(eng.ctx, reset=True)
    dx.dexel_profile_enable(eng.ctx, True)
    for _ in range(args.steps):
        for p in plans:
            p.enqueue()
    torch.cuda.synchronize()
    dx.dexel_profile_enable(eng.ctx, False)
    prof_ms, passes = dx.dexel_profile_read(eng.ctx, reset=True)

    ms_per_step = (t_end - t_start) * 1000.0 / args.steps
    n_in_step = sum(p.nseg_in for p in plans)
    value = n_in_step / (ms_per_step / 1000.0)
    per_step = {s_: prof_ms[i] / args.steps for i, s_ in enumerate(dx.PROFILE_STAGES)}
    roofline = stage_roofline(dx, per_step, pass_stats, ncols)
    kname = roofline["kernel"]
    traffic = measured_traffic(kname) if args.workload == "c3" else None
    roofline["traffic"] = int(traffic) if traffic is not None else None
    roofline.update(step_roofline(pass_stats, ncols, ms_per_step))
    roofline["copy_GBs_measured"] = measure_copy_gbs(torch)

    line = {
        "metric": "input dexel segments offset/sec",
        "value": value,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": float(np.median(step_ms)),
        "ms_per_step_min_max": [float(np.min(step_ms)), float(np.max(step_ms))],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "grid": f"{grid.nx}x{grid.ny}",
                   "nseg_in": grid.nseg, "ops": [f"{op} r={r}" for op, r in wl["ops"]],
                   "nseg_out": [p.nseg_out for p in plans]},
        "roofline": roofline,
        "kernels_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "variants": variants,
        "pass_sizes": [dict(st, nseg_in=n) for n, st in pass_stats],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(grid, wl["ops"], args.cpu_budget)
    print(json.dumps(line), flush=True)
    eng.close()


if __name__ == "__main__":
    main()
