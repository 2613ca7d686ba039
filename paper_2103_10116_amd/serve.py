"""Serving loop: a stream of independent SPD solves, continuous batching.

Requests arrive at given times (seconds after the start).  In "batched" mode
every arrived request is submitted to the libmxs batch engine, which admits
it into a free slot of its size class as soon as its footprint fits the HBM
budget, so new requests join while others are still iterating on the GPU.
In "plain" mode the same stream is served one request at a time by the
single-system CG (mxs_solve).  Latency of a request is completion time minus
arrival time on the host's monotonic clock.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I


@dataclass
class ServeReport:
    mode: str
    count: int
    wall_s: float                 # first arrival to last completion
    solves_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    iters_median: float
    statuses: dict
    steps: int = 0
    max_active: int = 0
    latencies_ms: np.ndarray = field(default=None, repr=False)
    x: dict = field(default=None, repr=False)

    def summary(self) -> dict:
        d = {k: getattr(self, k) for k in ("mode", "count", "wall_s", "solves_per_s", "p50_ms",
                                            "p99_ms", "mean_ms", "iters_median", "statuses",
                                            "steps", "max_active")}
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}


def build_systems(reqs):
    """(A, b) of every request, from its seed."""
    out = {}
    for r in reqs:
        A = I.serving_system(r.m, r.seed)
        out[r.rid] = (A, I.serving_rhs(A.n, r.seed))
    return out


def _report(mode, reqs, arrival, done, iters, statuses, t_first, keep_x, xs, steps=0,
            max_active=0):
    lat = np.array([done[r.rid] - arrival[r.rid] for r in reqs]) * 1e3
    wall = max(done.values()) - t_first
    st = {}
    for s in statuses.values():
        st[int(s)] = st.get(int(s), 0) + 1
    return ServeReport(mode, len(reqs), wall, len(reqs) / wall, float(np.percentile(lat, 50)),
                       float(np.percentile(lat, 99)), float(lat.mean()),
                       float(np.median(list(iters.values()))), st, steps, max_active, lat,
                       xs if keep_x else None)


def run_batched(ctx, reqs, systems, tol=1e-10, budget_bytes=2 << 30, max_slots=1024,
                iters_per_step=16, classes=None, staging_bytes=0, mode="f64",
                keep_x=False, chunk=512) -> ServeReport:
    """Continuous batching.  A submitter thread hands arrived requests to the
    engine (at most `chunk` per call) while the main thread steps: the host's
    validation and packing of new requests overlaps the device's steps, and
    requests join the batch at the next step after they are queued.  The
    main thread launches a step, then collects the results that earlier
    steps retired while it runs, then waits for it: the copying out of
    results overlaps the device too."""
    from . import mxs
    B = mxs.Batch(ctx, budget_bytes, max_slots, iters_per_step, classes, staging_bytes)
    order = sorted(reqs, key=lambda r: r.arrival)
    rid_of = {}
    arrival, done, iters, statuses, xs = {}, {}, {}, {}, {}
    lock = threading.Lock()
    failure = []
    queued = [0]
    t0 = time.perf_counter()

    def submitter():
        i = 0
        try:
            while i < len(order):
                now = time.perf_counter() - t0
                if order[i].arrival > now:
                    time.sleep(order[i].arrival - now)
                    continue
                j = i
                while j < len(order) and j - i < chunk and order[j].arrival <= now:
                    j += 1
                arrived = order[i:j]
                tickets, sts = B.submit_many([systems[r.rid] for r in arrived], tol, mode=mode)
                with lock:
                    for r, t, s in zip(arrived, tickets.tolist(), sts.tolist()):
                        if s != mxs.OK:
                            raise mxs.MxsError(s, f"request {r.rid} rejected")
                        rid_of[t] = r
                        arrival[r.rid] = r.arrival
                    queued[0] = j
                i = j
        except BaseException as e:  # reported by the stepping thread
            failure.append(e)

    th = threading.Thread(target=submitter, daemon=True)
    th.start()
    steps = 0
    max_active = 0
    early = []   # retired, not yet collected (or not yet recorded by the submitter)
    while len(done) < len(order):
        if failure:
            th.join()
            B.close()
            raise failure[0]
        with lock:
            work = queued[0] > len(done) + len(early)
        if work:
            B.step_launch()
            steps += 1
        with lock:
            ready = [t for t in early if t in rid_of]
            early = [t for t in early if t not in rid_of]
            rs = [rid_of[t] for t in ready]
        if ready:
            ns = [systems[r.rid][0].n for r in rs]
            sts, xbuf, off, info = B.poll_many(ready, ns)
            now = time.perf_counter() - t0
            for r, s, it, o, n in zip(rs, sts.tolist(), info["iters"].tolist(), off.tolist(), ns):
                done[r.rid] = now
                iters[r.rid] = it
                statuses[r.rid] = s
                if keep_x:
                    xs[r.rid] = xbuf[o:o + n]
        if work:
            st = B.step_finish()
            max_active = max(max_active, st["active"])
            early.extend(B.completed())
        elif not ready:
            time.sleep(50e-6)
    th.join()
    B.close()
    return _report("batched" if mode == "f64" else f"batched_{mode}", order, arrival, done,
                   iters, statuses, order[0].arrival, keep_x, xs, steps, max_active)


def run_plain(ctx, reqs, systems, tol=1e-10, keep_x=False) -> ServeReport:
    """One request at a time: upload, single-system CG, download."""
    import torch
    from . import mxs
    order = sorted(reqs, key=lambda r: r.arrival)
    arrival, done, iters, statuses, xs = {}, {}, {}, {}, {}
    t0 = time.perf_counter()
    for r in order:
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        A, b = systems[r.rid]
        M = mxs.Matrix.from_host(ctx, A)
        bd = torch.from_numpy(b).cuda()
        x = torch.zeros_like(bd)
        res = mxs.solve(ctx, "cg", M, bd, x, tol=tol, raise_on_error=False)
        xh = x.cpu().numpy()
        M.close()
        done[r.rid] = time.perf_counter() - t0
        arrival[r.rid] = r.arrival
        iters[r.rid] = res.iters
        statuses[r.rid] = res.status
        if keep_x:
            xs[r.rid] = xh
    return _report("plain", order, arrival, done, iters, statuses, order[0].arrival, keep_x, xs)
