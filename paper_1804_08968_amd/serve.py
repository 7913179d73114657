"""Continuous-batching offset server on one GPU.

Requests (op, radius, input shape or the previous result of the same
session) arrive over time.  The server keeps every shape and every session
result resident on the device, admits waiting requests into a batch while
their HBM footprint (input, output, workspace share) fits the free budget,
and keeps up to `slots` batches in flight on separate HIP streams, so work
of newly arrived requests overlaps with work already on the device.  A
chained request (open/close on the previous result of its session) becomes
eligible once that result is complete.  Completion times come from HIP
events, relative to an event recorded when the server starts.

Admission order (continuous mode, policy="sjf"): among the requests that are
the earliest waiting one of their session, smallest estimated work first,
with the estimate divided by 1 + wait / age_s so that a long-waiting large
request is eventually admitted.  The work estimate is (input intervals +
columns) x (1 + r), the row window the kernels walk per column.
policy="fifo" admits in arrival order.

mode="plain" serves one request at a time in arrival order with a
single-item call on one stream (the comparison point).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import torch

from . import (DEXEL_OK, DeviceGrid, Engine, OPS, dexel_batch_offset, dexel_batch_workspace_size,
               dexel_batch_item, make_out)


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the server start
    shape: int              # index into the shape pool (ignored for chained requests)
    op: str
    r: float
    chain: bool = False     # input = previous result of the same session
    session: int = 0


@dataclass
class Done:
    id: int
    arrival: float
    start: float            # host time the request's batch was enqueued
    done: float             # device completion time
    nseg_in: int
    status: int
    batch: int
    result: DeviceGrid | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    def __init__(self, engine: Engine, pool, budget_bytes: int = 64 << 30, max_batch: int = 16,
                 slots: int = 2, mode: str = "continuous", work_cap_cols: int = 4 << 20,
                 policy: str = "sjf", age_s: float = 2.0):
        self.engine = engine
        self.pool = list(pool)
        self.budget = int(budget_bytes)
        self.mode = mode
        if policy not in ("sjf", "fifo"):
            raise ValueError(f"unknown admission policy {policy!r}")
        self.policy = "fifo" if mode == "plain" else policy
        self.age_s = float(age_s)
        self.max_batch = 1 if mode == "plain" else int(max_batch)
        self.slots = 1 if mode == "plain" else int(slots)
        # A batch holds at most this many columns (one request always fits):
        # a request that fills the GPU on its own gains nothing from company,
        # and small requests should not wait for a large one to finish.
        self.work_cap = int(work_cap_cols)
        self.streams = [torch.cuda.Stream(device=engine.device) for _ in range(self.slots)]
        self.ws = [None] * self.slots   # per-slot workspace, grown on demand
        self.rejected = 0

    # -- footprint -----------------------------------------------------------
    def _item(self, grid: DeviceGrid, r: float, op: str, cap: int):
        dev = self.engine.device
        out = (torch.empty(grid.nx * grid.ny + 1, dtype=torch.int64, device=dev),
               torch.empty(2 * max(cap, 1), dtype=torch.float32, device=dev),
               torch.zeros(1, dtype=torch.int64, device=dev),
               torch.zeros(1, dtype=torch.int32, device=dev))
        it = dexel_batch_item()
        it.in_ = grid.view(grid.nseg_cached)
        it.r = float(r)
        it.op = OPS[op]
        it.out = make_out(grid.nx, grid.ny, out[0], out[1], out[2], out[3])
        return it, out

    @staticmethod
    def _out_cap(grid: DeviceGrid) -> int:
        return grid.nseg_cached + grid.nx * grid.ny + 1024

    def footprint(self, grid: DeviceGrid, r: float, op: str) -> int:
        view = grid.view(grid.nseg_cached)
        it = dexel_batch_item()
        it.in_ = view
        it.r = float(r)
        it.op = OPS[op]
        # this request's own default capacity, not the engine-wide retry hint
        ws = dexel_batch_workspace_size(self.engine.ctx, [it], 0)
        out = 8 * (grid.nx * grid.ny + 1) + 8 * self._out_cap(grid)
        return ws + out

    # -- main loop -----------------------------------------------------------
    def run(self, requests, poll_s: float = 2e-4):
        eng = self.engine
        for g in self.pool:
            if not hasattr(g, "nseg_cached"):
                g.nseg_cached = g.nseg
        reqs = sorted(requests, key=lambda q: q.arrival)
        pending = collections.deque(reqs)
        waiting: list[Request] = []
        inflight = []          # dicts: slot, event, members, mem, batch, ws
        free_slots = list(range(self.slots))
        session_last: dict[int, DeviceGrid] = {}
        session_busy: set[int] = set()
        results: dict[int, Done] = {}
        used = 0
        batch_id = 0
        torch.cuda.synchronize(eng.device)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        torch.cuda.synchronize(eng.device)
        t0 = time.perf_counter()

        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # retire finished batches (their inputs for chained requests are then complete)
            still = []
            for b in inflight:
                if not b["event"].query():
                    still.append(b)
                    continue
                done_t = ref.elapsed_time(b["event"]) / 1000.0
                for req, grid_in, out, start in b["members"]:
                    st = int(out[3].item())
                    res = DeviceGrid(grid_in.nx, grid_in.ny, out[0], out[1])
                    t_done = done_t
                    if st != DEXEL_OK:
                        # rare: output or workspace too small; redo alone, synchronously
                        res = eng.offset(grid_in, req.r, req.op)
                        t_done = time.perf_counter() - t0
                        st = DEXEL_OK
                    res.nseg_cached = int(res.col_ptr[-1].item())
                    session_last[req.session] = res
                    session_busy.discard(req.session)
                    results[req.id] = Done(req.id, req.arrival, start, t_done,
                                           grid_in.nseg_cached, st, b["batch"], res)
                used -= b["mem"]
                free_slots.append(b["slot"])
            inflight = still
            # admit waiting requests into a new batch on a free slot
            launched = False
            if free_slots and waiting:
                members, mem_b, keep = [], 0, []
                cols_b = 0
                held = set()           # sessions with an earlier request still waiting
                order = waiting
                if self.policy == "sjf":
                    first = {}
                    for req in waiting:    # waiting is in arrival order
                        first.setdefault(req.session, req.id)

                    def prio(req):
                        g = (session_last.get(req.session, self.pool[req.shape]) if req.chain
                             else self.pool[req.shape])
                        work = (g.nseg_cached + g.nx * g.ny) * (1.0 + req.r)
                        return work / (1.0 + (now - req.arrival) / self.age_s)
                    heads = sorted((q for q in waiting if first[q.session] == q.id), key=prio)
                    order = heads + [q for q in waiting if first[q.session] != q.id]
                for req in order:
                    if (len(members) >= self.max_batch or req.session in session_busy
                            or req.session in held):
                        keep.append(req)   # full batch, or keep the session's order
                        held.add(req.session)
                        continue
                    if req.chain and req.session in session_last:
                        grid_in = session_last[req.session]
                    else:
                        grid_in = self.pool[req.shape]
                    fp = self.footprint(grid_in, req.r, req.op)
                    if fp > self.budget:
                        self.rejected += 1
                        results[req.id] = Done(req.id, req.arrival, now, now, grid_in.nseg_cached,
                                               -4, -1, None)
                        continue
                    if used + mem_b + fp > self.budget or (
                            members and cols_b + grid_in.nx * grid_in.ny > self.work_cap):
                        keep.append(req)   # waits until memory or batch room frees up
                        held.add(req.session)
                        continue
                    members.append((req, grid_in))
                    mem_b += fp
                    cols_b += grid_in.nx * grid_in.ny
                    session_busy.add(req.session)
                waiting = sorted(keep, key=lambda q: (q.arrival, q.id))
                if members:
                    slot = free_slots.pop()
                    stream = self.streams[slot]
                    items, outs = [], []
                    for req, grid_in in members:
                        it, out = self._item(grid_in, req.r, req.op, self._out_cap(grid_in))
                        items.append(it)
                        outs.append(out)
                    nbytes = dexel_batch_workspace_size(eng.ctx, items, 0)
                    ws = self.ws[slot]
                    if ws is None or ws.numel() < nbytes:
                        self.ws[slot] = None
                        with torch.cuda.stream(stream):
                            ws = torch.empty(int(nbytes * 1.25), dtype=torch.uint8,
                                             device=eng.device)
                        self.ws[slot] = ws
                    # the outputs were allocated and zeroed on the current stream
                    stream.wait_stream(torch.cuda.current_stream(eng.device))
                    st = dexel_batch_offset(eng.ctx, items, ws, stream, 0)
                    if st != DEXEL_OK:
                        raise RuntimeError(f"batch enqueue failed with status {st}")
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(stream)
                    start = time.perf_counter() - t0
                    used += mem_b
                    inflight.append({"slot": slot, "event": ev, "mem": mem_b, "batch": batch_id,
                                     "ws": ws, "items": items,
                                     "members": [(req, grid_in, out, start)
                                                 for (req, grid_in), out in zip(members, outs)]})
                    batch_id += 1
                    launched = True
            if not launched and not (pending and pending[0].arrival <= time.perf_counter() - t0):
                time.sleep(poll_s)
        return [results[q.id] for q in reqs]


def summarize(done, t_makespan=None):
    """Latency percentiles (ms) and throughput of a served stream."""
    import numpy as np
    ok = [d for d in done if d.status == 0]
    lat = np.array([d.latency for d in ok]) * 1000.0
    span = t_makespan if t_makespan is not None else (
        max(d.done for d in ok) - min(d.arrival for d in ok) if ok else 0.0)
    segs = sum(d.nseg_in for d in ok)
    return {
        "requests": len(done), "completed": len(ok), "rejected": len(done) - len(ok),
        "latency_ms_p50": float(np.percentile(lat, 50)) if ok else None,
        "latency_ms_p99": float(np.percentile(lat, 99)) if ok else None,
        "latency_ms_mean": float(lat.mean()) if ok else None,
        "segments_per_s": segs / span if span > 0 else None,
        "batches": len({d.batch for d in ok}),
        "makespan_s": span,
    }
