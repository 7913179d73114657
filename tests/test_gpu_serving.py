"""Serving: the same requests give the same results alone (plain server, one
request at a time) and in the mix (continuous batching, several batches in
flight, chained requests on device-resident session state), bit for bit,
equal to the oracle's float32 model replayed session by session, and within
tolerance of the float64 oracle applied to each request's own input."""
from __future__ import annotations

import numpy as np
import pytest

from synth import gen
from tests.helpers import compare_columns, random_grid

pytestmark = pytest.mark.gpu


def _pool(dx):
    rng = np.random.default_rng(12)
    hosts = [random_grid(rng, int(rng.integers(20, 90)), int(rng.integers(20, 90)), 80.0,
                         max_per_col=5) for _ in range(4)]
    hosts.append(gen.gyroid_grid(1, n=64, height=96.0, period=24.0, t=0.35))
    hosts.append(gen.spheres_grid(2, n=72, count=7))
    return hosts, [dx.DeviceGrid.from_host(h) for h in hosts]


def _requests(serve, n, rate, seed):
    """Same requests for every rate; arrivals (all at 0, or Poisson at
    `rate` per second) come from a separate generator."""
    rng = np.random.default_rng(seed)
    arr = np.random.default_rng(seed + 1000)
    ops = ["dilate", "erode", "open", "close"]
    t, out = 0.0, []
    for i in range(n):
        t += 0.0 if rate is None else arr.exponential(1.0 / rate)
        out.append(serve.Request(i, t, int(rng.integers(0, 6)), ops[int(rng.integers(0, 4))],
                                 float(rng.uniform(1.0, 6.0)), bool(rng.random() < 0.3),
                                 int(rng.integers(0, 7))))
    return out


def _host(dg):
    cp, z = dg.to_host()
    return cp.copy(), z.astype(np.float64).copy()


def test_alone_equals_mix(engine, oracle_lib):
    import paper_1804_08968_amd as dx
    from paper_1804_08968_amd import serve
    hosts, pool = _pool(dx)
    reqs = _requests(serve, 36, None, 3)
    print("[case] plain", flush=True)
    plain = serve.Server(engine, pool, mode="plain").run(reqs)
    print("[case] continuous burst", flush=True)
    burst = serve.Server(engine, pool, max_batch=8, slots=3).run(reqs)
    timed = _requests(serve, 36, 400.0, 3)
    print("[case] continuous poisson", flush=True)
    pois = serve.Server(engine, pool, max_batch=8, slots=2).run(timed)
    assert max(d.batch for d in burst) < len(reqs) - 1  # requests were really batched
    for a, b, c in zip(plain, burst, pois):
        assert a.status == b.status == c.status == 0
        ha, hb, hc = _host(a.result), _host(b.result), _host(c.result)
        assert np.array_equal(ha[0], hb[0]) and np.array_equal(ha[1], hb[1]), a.id
        assert np.array_equal(ha[0], hc[0]) and np.array_equal(ha[1], hc[1]), a.id
    # oracle replay per session (float32 model, intermediate results rounded to float32)
    last = {}
    for q, d in zip(reqs, plain):
        src = last[q.session] if (q.chain and q.session in last) else oracle_lib.Grid.from_any(hosts[q.shape])
        ref = oracle_lib.run(src, q.r, q.op, "f32model")
        last[q.session] = ref
        cp, z = _host(d.result)
        assert np.array_equal(cp, ref.col_ptr) and np.array_equal(z, ref.z), q
        # and within tolerance of the float64 oracle on the same input
        ref64 = oracle_lib.run(src, q.r, q.op, "f64")
        res = compare_columns(np.diff(ref64.col_ptr), ref64.z, np.diff(cp), z, q.r,
                              k=2 if q.op in ("open", "close") else 1)
        assert res["failed"] == 0, (q, res)


def test_admission_rejects_oversized(engine):
    import paper_1804_08968_amd as dx
    from paper_1804_08968_amd import serve
    _, pool = _pool(dx)
    reqs = _requests(serve, 6, None, 5)
    done = serve.Server(engine, pool, budget_bytes=1024).run(reqs)
    assert all(d.status == -4 for d in done)
    summary = serve.summarize(done)
    assert summary["completed"] == 0 and summary["rejected"] == 6


def test_admission_counts_held_memory(engine):
    """The budget covers slot workspaces and every output still held: at the
    end of a run the server holds exactly its slot workspaces plus every
    result (keep_results) or each session's last result (otherwise).  With
    results dropped as their session moves on, a budget of about two
    requests' footprint serves the whole stream without passing it."""
    import paper_1804_08968_amd as dx
    from paper_1804_08968_amd import serve
    _, pool = _pool(dx)
    reqs = _requests(serve, 12, None, 7)
    probe = serve.Server(engine, pool)
    for g in pool:
        g.nseg_cached = g.nseg
    fps = [probe.footprint(pool[q.shape], q.r, q.op) for q in reqs if not q.chain]
    budget = int(2.6 * max(fps))
    print(f"[case] serving budget {budget}", flush=True)
    for keep in (False, True):
        srv = serve.Server(engine, pool, budget_bytes=budget, max_batch=4, slots=2, keep_results=keep)
        done = srv.run(reqs)
        ok = [d for d in done if d.status == 0]
        assert all(d.status in (0, -4) for d in done)
        assert 0 < srv.peak_bytes <= budget
        ws = sum(w.numel() for w in srv.ws if w is not None)
        if keep:
            held = sum(serve.Server._grid_bytes(d.result) for d in ok)
            assert srv.held_bytes == ws + held, (srv.held_bytes, ws, held)
        else:
            # every request served; only the sessions' last results stay
            assert len(ok) == len(done) and all(d.result is None for d in done)
            assert ws < srv.held_bytes <= srv.peak_bytes
