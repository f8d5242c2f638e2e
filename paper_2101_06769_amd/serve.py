"""Serving loop: independent solves admitted over time and advanced together.

Requests (a case, its initial fields and a number of steps) arrive over time.
The continuous-batching server admits them in arrival order while its
device-memory budget and a batch slot allow. Each admitted state stays
resident in HBM. All admitted solves advance in the same batched
launches (graph-replayed chunks of steps). A request that arrives while
others run joins at the next step boundary. A finished solve is read back
(phi, u, p), detached, and its memory returned to the budget.

The baseline server runs one request at a time to completion, in arrival
order, each as a plain solver with its own launches.

A solve whose state turns non-finite is retired after the quantum in which
the batch flagged it, and reported unstable.

Every device operation goes through the C ABI (``mplb``). This module only
schedules. Latency is measured from a request's arrival to its result being
on the host, on a clock that starts when the replay starts.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import inputs, mplb


@dataclasses.dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    cells: int
    status: int
    fields: dict | None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def _case_of(spec):
    return spec["case"] if "case" in spec else inputs.serving_case(spec)


def _arena_bytes(case, storage):
    return mplb.state_bytes(mplb.make_params(case.params, storage)) + 256


class _Replay:
    """Arrival clock: requests become visible when the wall clock passes
    their arrival time (realtime), or all at once (as fast as possible)."""

    def __init__(self, specs, realtime):
        self.pending = collections.deque(sorted(specs, key=lambda s: s["arrival"]))
        self.realtime = realtime
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def arrived(self):
        """Requests visible now, each with its arrival time on the replay
        clock (the scheduled time in real time, else the time it was seen)."""
        out = []
        t = self.now()
        while self.pending and (not self.realtime or self.pending[0]["arrival"] <= t):
            spec = dict(self.pending.popleft())
            if not self.realtime:
                spec["arrival"] = t
            out.append(spec)
        return out

    def wait_next(self):
        if self.pending and self.realtime:
            dt = self.pending[0]["arrival"] - self.now()
            if dt > 0:
                time.sleep(dt)


def _finish(solver, keep_fields):
    red, rc = solver.reduce()
    f = solver.fields() if keep_fields else None
    return rc, f


def serve_batched(specs, dim=2, storage="fp32", hbm_budget=8 << 30, capacity=64, quantum=64,
                  chunk=16, realtime=True, keep_fields=False, block=(128, 2, 1), on_event=None):
    """Continuous batching. Returns (results, stats). stats holds the peak
    device bytes admitted, the peak number of concurrent solves and the
    batch steps taken.  The batch advances `quantum` steps between
    admission / completion checks (a finished solve waits at most that long
    to be collected; a new one at most that long to join)."""
    import torch

    batch = mplb.Batch(dim, storage, capacity=capacity, max_tiles=1 << 22)
    batch.set_graph_chunk(chunk)
    if block is not None:
        batch.set_block(*block)
    rp = _Replay(specs, realtime)
    queue = collections.deque()
    active = {}  # slot -> (spec, solver, nbytes, admitted time, cells)
    used = peak_used = peak_active = 0
    results = []
    rejected = []
    while rp.pending or queue or active:
        for spec in rp.arrived():
            case = _case_of(spec)
            queue.append((spec, case, _arena_bytes(case, storage)))
        # admission, in arrival order (head of line)
        while queue and len(active) < capacity:
            spec, case, need = queue[0]
            if need > hbm_budget:  # can never fit: reject now
                queue.popleft()
                rejected.append(spec["id"])
                results.append(Result(spec["id"], spec["arrival"], rp.now(), rp.now(),
                                      spec["steps"], case.ncells, mplb.ENOMEM, None))
                continue
            if used + need > hbm_budget:
                break
            queue.popleft()
            s = mplb.Solver(case.params, storage=storage, stream=batch.stream)
            s.init(case.phi, case.u, case.p)
            slot = batch.attach(s, spec["steps"])
            used += need
            active[slot] = (spec, s, need, rp.now(), case.ncells)
            peak_used = max(peak_used, used)
            peak_active = max(peak_active, len(active))
            if on_event:
                on_event("admit", spec["id"], len(active), used)
        if not active:
            rp.wait_next()
            continue
        # a full quantum: a solve whose window closes inside it stops at its
        # own last step (the batch skips it), and is collected after
        batch.step(quantum)
        # a solve whose state went non-finite is retired at once (the batch
        # flags it during the quantum and closes its window): its slot and
        # memory go back to the queue instead of running out its steps
        status = batch.status()
        for sl in [sl for sl in active if status.get(sl) == mplb.EUNSTABLE]:
            spec, s, need, t_adm, cells = active.pop(sl)
            batch.detach(sl)
            results.append(Result(spec["id"], spec["arrival"], t_adm, rp.now(), spec["steps"],
                                  cells, mplb.EUNSTABLE, None))
            used -= need
            del s
            if on_event:
                on_event("unstable", spec["id"], len(active), used)
        for sl in [sl for sl in active if batch.remaining(sl) == 0]:
            spec, s, need, t_adm, cells = active.pop(sl)
            batch.detach(sl)
            rc, f = _finish(s, keep_fields)
            results.append(Result(spec["id"], spec["arrival"], t_adm, rp.now(), spec["steps"],
                                  cells, rc, f))
            used -= need
            del s
            if on_event:
                on_event("finish", spec["id"], len(active), used)
    torch.cuda.synchronize()
    results.sort(key=lambda r: r.id)
    return results, dict(peak_bytes=peak_used, peak_active=peak_active,
                         batch_steps=batch.steps_done(), rejected=rejected)


def serve_fifo(specs, storage="fp32", realtime=True, keep_fields=False):
    """Baseline: one request at a time, to completion, in arrival order,
    each a plain solver with its own launches."""
    import torch

    rp = _Replay(specs, realtime)
    queue = collections.deque()
    results = []
    while rp.pending or queue:
        queue.extend(rp.arrived())
        if not queue:
            rp.wait_next()
            continue
        spec = queue.popleft()
        case = _case_of(spec)
        t_adm = rp.now()
        s = mplb.Solver(case.params, storage=storage)
        s.init(case.phi, case.u, case.p)
        s.step(spec["steps"])
        rc, f = _finish(s, keep_fields)
        results.append(Result(spec["id"], spec["arrival"], t_adm, rp.now(), spec["steps"],
                              case.ncells, rc, f))
        del s
    torch.cuda.synchronize()
    results.sort(key=lambda r: r.id)
    return results


def summary(results, wall):
    """p50 / p99 latency (s), jobs/s and aggregate MLUPS of a replay."""
    lat = np.array([r.latency for r in results if r.status == mplb.OK])
    ok = len(lat)
    work = sum(r.cells * r.steps for r in results if r.status == mplb.OK)
    return dict(jobs=len(results), ok=ok,
                p50_s=float(np.percentile(lat, 50)) if ok else None,
                p99_s=float(np.percentile(lat, 99)) if ok else None,
                jobs_per_s=ok / wall if wall > 0 else None,
                mlups=work / wall / 1e6 if wall > 0 else None)
