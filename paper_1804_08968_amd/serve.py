"""Continuous-batching offset server on one GPU.

Requests (op, radius, input shape or the previous result of the same
session) arrive over time.  The server keeps every shape and every session
result resident on the device, admits waiting requests into a batch while
the device memory the batch adds fits the budget, and keeps up to `slots`
batches in flight on separate HIP streams, so work
of newly arrived requests overlaps with work already on the device.  A
chained request (open/close on the previous result of its session) becomes
eligible once that result is complete.  Completion times come from HIP
events, relative to an event recorded when the server starts.

Admission order (continuous mode): policy="fifo" (the default) takes the
waiting requests in arrival order and admits each that fits; one that does
not (memory, or the columns the batches in flight already hold) waits while
later ones that fit go ahead of it (backfill).  policy="sjf" takes, among
the requests that are the earliest waiting one of their session, the
smallest estimated work first, with the estimate divided by 1 + wait / age_s
so that a long-waiting large request is eventually admitted; the work
estimate is (input intervals + columns) x (1 + r), the row window the
kernels walk per column.  SJF gives the lower median, FIFO with backfill the
shorter tail (large requests are not passed indefinitely).

mode="plain" serves one request at a time in arrival order with a
single-item call on one stream (the comparison point).

Memory accounting: the budget covers what the server holds on the device
beyond the shape pool: each slot's workspace (kept, and grown on demand to
1.25 x the batch that needed it) and every output buffer from the admission
of its request until it is dropped.  An output is dropped when a later
request of the same session replaces it as the session's result, unless
keep_results is set (then every result is returned to the caller and held
until the run ends).  A batch is admitted if the outputs of its members
plus the growth of its slot's workspace (the members' single-item
workspaces summed, an upper bound of the batch's) fit in what is free; a
request that cannot fit even with nothing in flight is rejected (status
DEXEL_ERR_WORKSPACE).
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
                 policy: str = "fifo", age_s: float = 2.0, keep_results: bool = True):
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
        # The batches in flight hold at most this many columns together (one
        # request always fits when nothing else is in flight): a request that
        # fills the GPU on its own gains nothing from company, small requests
        # should not wait for a large one to finish, and two large requests
        # sharing the GPU would each take about twice as long.
        self.work_cap = int(work_cap_cols)
        self.streams = [torch.cuda.Stream(device=engine.device) for _ in range(self.slots)]
        self.ws = [None] * self.slots   # per-slot workspace, grown on demand
        self.keep_results = bool(keep_results)
        self.rejected = 0
        self.peak_bytes = 0     # most device bytes held at once (the budget's measure)
        self.held_bytes = 0

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

    @staticmethod
    def _out_bytes(grid: DeviceGrid) -> int:
        """Device bytes of one request's output CSR buffers (its two status
        scalars aside)."""
        return 8 * (grid.nx * grid.ny + 1) + 8 * Server._out_cap(grid)

    @staticmethod
    def _grid_bytes(g: DeviceGrid) -> int:
        return 8 * g.col_ptr.numel() + 4 * g.z.numel()

    def _ws_bytes(self, grid: DeviceGrid, r: float, op: str) -> int:
        """Single-item workspace of a request, at its own default capacity
        (not the engine-wide retry hint)."""
        it = dexel_batch_item()
        it.in_ = grid.view(grid.nseg_cached)
        it.r = float(r)
        it.op = OPS[op]
        return dexel_batch_workspace_size(self.engine.ctx, [it], 0)

    def footprint(self, grid: DeviceGrid, r: float, op: str) -> int:
        """Device bytes a request adds when served alone: its output and a
        workspace sized for it."""
        return self._ws_bytes(grid, r, op) + self._out_bytes(grid)

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
        session_bytes: dict[int, int] = {}   # device bytes of each session's result buffers
        session_busy: set[int] = set()
        results: dict[int, Done] = {}
        # device bytes held beyond the pool: slot workspaces and live outputs
        used = sum(w.numel() for w in self.ws if w is not None)
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
                    nbytes = self._out_bytes(grid_in)
                    t_done = done_t
                    if st != DEXEL_OK:
                        # rare: output or workspace too small; redo alone, synchronously
                        res = eng.offset(grid_in, req.r, req.op)
                        used += self._grid_bytes(res) - nbytes
                        nbytes = self._grid_bytes(res)
                        t_done = time.perf_counter() - t0
                        st = DEXEL_OK
                    res.nseg_cached = int(res.col_ptr[-1].item())
                    if not self.keep_results:
                        # the result it replaces is no longer referenced
                        used -= session_bytes.get(req.session, 0)
                    session_last[req.session] = res
                    session_bytes[req.session] = nbytes
                    session_busy.discard(req.session)
                    results[req.id] = Done(req.id, req.arrival, start, t_done,
                                           grid_in.nseg_cached, st, b["batch"],
                                           res if self.keep_results else None)
                free_slots.append(b["slot"])
            inflight = still
            # admit waiting requests into a new batch on a free slot
            launched = False
            if free_slots and waiting:
                members, mem_b, keep = [], 0, []
                cols_b, ws_b = 0, 0
                cols_busy = sum(b["cols"] for b in inflight)
                slot_ws = self.ws[free_slots[-1]]
                slot_have = slot_ws.numel() if slot_ws is not None else 0
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
                    out_b = self._out_bytes(grid_in)
                    w_b = self._ws_bytes(grid_in, req.r, req.op)
                    grow = max(0, int((ws_b + w_b) * 1.25) - slot_have)
                    if not inflight and not members and used + out_b + grow > self.budget:
                        # nothing in flight: the slots' workspaces are idle and can go
                        idle = sum(w.numel() for w in self.ws if w is not None)
                        if used - idle + out_b + int(w_b * 1.25) <= self.budget:
                            self.ws = [None] * self.slots
                            used -= idle
                            slot_have = 0
                            grow = int(w_b * 1.25)
                    if (out_b + int(w_b * 1.25) > self.budget
                            or (not inflight and not members and used + out_b + grow > self.budget)):
                        # cannot fit, even with nothing else held but the results
                        self.rejected += 1
                        results[req.id] = Done(req.id, req.arrival, now, now, grid_in.nseg_cached,
                                               -4, -1, None)
                        continue
                    if used + mem_b + out_b + grow > self.budget or (
                            (members or inflight)
                            and cols_busy + cols_b + grid_in.nx * grid_in.ny > self.work_cap):
                        keep.append(req)   # waits until memory or GPU room frees up
                        held.add(req.session)
                        continue
                    members.append((req, grid_in))
                    mem_b += out_b
                    ws_b += w_b
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
                        used -= ws.numel() if ws is not None else 0
                        self.ws[slot] = ws = None
                        with torch.cuda.stream(stream):
                            ws = torch.empty(int(nbytes * 1.25), dtype=torch.uint8,
                                             device=eng.device)
                        self.ws[slot] = ws
                        used += ws.numel()
                    # the outputs were allocated and zeroed on the current stream
                    stream.wait_stream(torch.cuda.current_stream(eng.device))
                    st = dexel_batch_offset(eng.ctx, items, ws, stream, 0)
                    if st != DEXEL_OK:
                        raise RuntimeError(f"batch enqueue failed with status {st}")
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(stream)
                    start = time.perf_counter() - t0
                    used += mem_b  # the outputs; the workspace was counted as it grew
                    self.peak_bytes = max(self.peak_bytes, used)
                    inflight.append({"slot": slot, "event": ev, "mem": mem_b, "cols": cols_b,
                                     "batch": batch_id,
                                     "ws": ws, "items": items,
                                     "members": [(req, grid_in, out, start)
                                                 for (req, grid_in), out in zip(members, outs)]})
                    batch_id += 1
                    launched = True
            if not launched and not (pending and pending[0].arrival <= time.perf_counter() - t0):
                time.sleep(poll_s)
        self.held_bytes = used   # at the end: slot workspaces and the outputs still held
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
