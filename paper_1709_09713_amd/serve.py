"""Continuous-batching serving loop for independent Taylor-Green solves.

Requests (grid size, Reynolds and Mach numbers, time step, step count)
arrive over wall-clock time.  The server admits them first-come first-served
into a Batch as long as a slot is free and the sum of member footprints
(state + fused workspace) stays within an HBM budget, keeps every admitted
state resident on the device, and advances all members together in quanta
of a few RK3 steps.  Because step accounting is host-side, the server knows
which members finish in a quantum when it queues it: they are retired at
once, and their final diagnostics are read on a side stream as soon as that
quantum has run, while the next quantum is already queued.  The latency of a
request is arrival -> its final diagnostics on the host.

``serve_sequential`` is the comparison: the same requests solved one at a
time, first come first served, with rk3_step.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as nat
from .batch import Batch


@dataclass
class Result:
    rid: int
    n: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    diag: dict = field(default_factory=dict)
    state: object = None

    @property
    def latency(self):
        return self.finished - self.arrival


def _points(req):
    n = req["n"]
    return n ** 3 if isinstance(n, int) else int(np.prod(n))


def summarize(results, t_first, t_last):
    """Latency percentiles, throughput, and two signs of whether the offered
    load was sustained: the requests still unfinished when the last one
    arrived (a queue that keeps growing leaves a backlog proportional to the
    run length) and the mean latency of the last quarter of arrivals over
    that of the first quarter."""
    lat = np.array([r.latency for r in results])
    upd = sum(_points(dict(n=r.n)) * 3 * r.steps for r in results)
    span = t_last - t_first
    last_arrival = max(r.arrival for r in results)
    by_arrival = sorted(results, key=lambda r: r.arrival)
    q = max(1, len(by_arrival) // 4)
    first = np.mean([r.latency for r in by_arrival[:q]])
    last = np.mean([r.latency for r in by_arrival[-q:]])
    return {"requests": len(results),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "makespan_s": span,
            "updates_per_s": upd / span,
            "requests_per_s": len(results) / span,
            "backlog_at_last_arrival": int(sum(r.finished > last_arrival for r in results)),
            "latency_last_over_first_quarter": float(last / first) if first > 0 else None}


class GpuBackend:
    """What the server needs from the device: a batch, stream events, a
    side stream, final diagnostics and member footprints."""

    def __init__(self, precision: str, max_instances: int, nstreams: int):
        self.precision = precision
        self.max_instances = max_instances
        self.nstreams = nstreams

    def stream(self):
        return torch.cuda.current_stream()

    def side_stream(self):
        return torch.cuda.Stream()

    def batch(self):
        return Batch(self.max_instances, self.precision, nstreams=self.nstreams)

    def event(self, stream):
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev

    def diagnostics(self, p, state, work, side, ev):
        side.wait_event(ev)
        return nat.diagnostics(p, state, work, stream=side)

    def footprint(self, n) -> int:
        return Batch.footprint(n, self.precision)

    def free_bytes(self) -> int:
        return torch.cuda.mem_get_info()[0]

    def host_state(self, state):
        return state.cpu().numpy()


class Server:
    """max_instances is the number of requests advanced together.  Once the
    members in flight fill the device, more of them only share it and
    stretch every request's latency, so the default is small: on the
    32^3..192^3 request mix four concurrent members gave both the lowest
    latency and the highest throughput (64 members: p50 +50%, throughput
    -4%)."""

    def __init__(self, precision: str = "fp32", max_instances: int = 4,
                 hbm_budget: int | None = None, nstreams: int = 3, quantum: int = 25,
                 tuner=None, keep_states: bool = False, backend=None):
        self.precision = precision
        self.max_instances = max_instances
        self.backend = backend or GpuBackend(precision, max_instances, nstreams)
        if hbm_budget is None:
            hbm_budget = min(32 << 30, self.backend.free_bytes() // 2)
        self.hbm_budget = hbm_budget
        self.nstreams = nstreams
        self.quantum = quantum
        self.tuner = tuner
        self.keep_states = keep_states

    def run(self, requests):
        """Serve `requests` (dicts with rid, arrival [s from start], n,
        reynolds, mach, dt, steps) in real time; returns (results sorted by
        rid, summary)."""
        if not requests:
            return [], {"requests": 0}
        be = self.backend
        stream = be.stream()
        side = be.side_stream()
        batch = be.batch()
        pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
        for r in pending:
            if be.footprint(r["n"]) > self.hbm_budget:
                raise ValueError(f"request {r['rid']} alone exceeds the HBM budget")
        active = {}     # slot -> [req, admitted, steps_left]
        draining = []   # (event, req, admitted, params, state, work)
        results = []
        used = 0
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def drain(force):
            # read the final diagnostics of retired members whose last
            # quantum has run (all of them with force), on the side stream
            nonlocal used
            keep = []
            for item in draining:
                ev, req, adm, p, state, work = item
                if force or ev.query():
                    d = be.diagnostics(p, state, work, side, ev)
                    res = Result(req["rid"], req["n"], req["steps"], req["arrival"], adm, now(), d)
                    if self.keep_states:
                        res.state = be.host_state(state)
                    results.append(res)
                    used -= be.footprint(req["n"])
                else:
                    keep.append(item)
            draining[:] = keep

        prev = None
        try:
            while pending or active or draining:
                # admission: first come first served, by free slot and footprint
                while (pending and pending[0]["arrival"] <= now()
                       and len(active) < self.max_instances):
                    req = pending[0]
                    fp = be.footprint(req["n"])
                    if used + fp > self.hbm_budget:
                        break
                    pending.popleft()
                    tile, zc = (self.tuner.lookup(req["n"], self.precision) if self.tuner
                                else (-1, 0))
                    slot = batch.add(req["n"], reynolds=req["reynolds"], mach=req["mach"],
                                     dt=req["dt"], steps=req["steps"], tile=tile, zchunk=zc,
                                     stream=stream)
                    active[slot] = [req, now(), req["steps"]]
                    used += fp
                if not active:
                    if draining:
                        drain(True)
                    elif pending:
                        time.sleep(max(0.0, pending[0]["arrival"] - now()))
                    continue
                q = min(self.quantum, min(a[2] for a in active.values()))
                batch.step(q, stream)
                ev = be.event(stream)
                for slot in list(active):
                    a = active[slot]
                    a[2] -= q
                    if a[2] == 0:
                        p, state, work = batch.remove(slot)
                        draining.append((ev, a[0], a[1], p, state, work))
                        del active[slot]
                # two quanta in flight: wait for the previous one only
                if prev is not None:
                    prev.synchronize()
                drain(False)
                prev = ev
        finally:
            batch.close()
        results.sort(key=lambda r: r.rid)
        t_first = min(r["arrival"] for r in requests)
        t_last = max(r.finished for r in results)
        return results, summarize(results, t_first, t_last)


def serve_sequential(requests, precision: str = "fp64", keep_states: bool = False):
    """The same requests solved one at a time, first come first served,
    each with one rk3_step call of the fused class."""
    if not requests:
        return [], {"requests": 0}
    stream = torch.cuda.current_stream()
    prec = nat.PRECS[precision]
    results = []
    t0 = time.perf_counter()
    for req in sorted(requests, key=lambda r: r["arrival"]):
        wait = req["arrival"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        adm = time.perf_counter() - t0
        n = req["n"]
        p = nat.make_params(n, reynolds=req["reynolds"], mach=req["mach"])
        nx, ny, nz = p.n
        state = torch.empty((5, nz, ny, nx), dtype=torch.float64, device="cuda")
        work = torch.empty(nat.ns_workspace_bytes(p, nat.NS_ALGO_FUSED, prec), dtype=torch.uint8,
                           device="cuda")
        nat.tgv_init(p, state, stream)
        nat.rk3_step(p, nat.NS_ALGO_FUSED, prec, req["dt"], req["steps"], state, work,
                     stream=stream)
        d = nat.diagnostics(p, state, work, stream=stream)
        res = Result(req["rid"], n, req["steps"], req["arrival"], adm, time.perf_counter() - t0, d)
        if keep_states:
            res.state = state.cpu().numpy()
        results.append(res)
    results.sort(key=lambda r: r.rid)
    t_first = min(r["arrival"] for r in requests)
    t_last = max(r.finished for r in results)
    return results, summarize(results, t_first, t_last)
