"""Continuous-batching request loop over the sparse spectral solver.

Requests (problems of any dimension, stamp size and precision) arrive over
time.  A builder thread pool builds each request's stamping set and operator
on its own HIP stream as soon as it arrives; built requests wait in a ready
queue; the scheduler admits them into a ``sparsespec.Engine`` whenever the
engine's slot count and HBM budget allow (the engine refuses a request that
would exceed them, and it stays queued), and advances every admitted problem
with shared launches, a few CG iterations per tick.  Requests that finish are
retired between ticks, which frees their slot and memory for the next ones, so
requests arriving while others are on the GPU join the running batch.

The scheduler core (``Scheduler``) only talks to an engine and a builder
through small interfaces, so its admission and accounting logic is tested on
the CPU with stand-ins.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Callable, Dict, List, Sequence

import numpy as np


@dataclasses.dataclass
class Finished:
    rid: int
    arrival: float
    admitted: float
    done: float
    info: dict
    result: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """Admission and retirement bookkeeping for one engine.

    ``engine`` must provide ``submit(handle, tag) -> bool`` (False when the
    budget or slots are exhausted), ``step(iters) -> n_active`` and
    ``poll() -> [(tag, prob, info)]``.  ``handle`` is whatever the builder made
    for a request; a request is finished when all ``n_prob`` of its problems
    have been polled.
    """

    def __init__(self, engine, iters_per_tick: int = 4, clock: Callable[[], float] = time.perf_counter):
        self.engine = engine
        self.iters = iters_per_tick
        self.clock = clock
        self.ready: collections.deque = collections.deque()      # (rid, arrival, handle, n_prob)
        self.active: Dict[int, list] = {}                          # rid -> [arrival, admitted, handle, left]
        self.finished: List[Finished] = []
        self.max_active = 0

    def offer(self, rid: int, arrival: float, handle, n_prob: int = 1):
        self.ready.append((rid, arrival, handle, n_prob))

    def admit(self) -> int:
        """Admit ready requests in arrival order until the engine refuses one."""
        n = 0
        while self.ready:
            rid, arrival, handle, n_prob = self.ready[0]
            if not self.engine.submit(handle, rid):
                break
            self.ready.popleft()
            self.active[rid] = [arrival, self.clock(), handle, n_prob]
            n += 1
        self.max_active = max(self.max_active, len(self.active))
        return n

    def tick(self) -> int:
        """One engine step plus retirement; returns the number of requests finished."""
        if not self.active:
            return 0
        self.engine.step(self.iters)
        done = 0
        for tag, prob, info in self.engine.poll():
            rec = self.active[tag]
            rec[3] -= 1
            if rec[3] == 0:
                arrival, admitted, handle, _ = self.active.pop(tag)
                self.finished.append(Finished(tag, arrival, admitted, self.clock(), info, handle))
                done += 1
        return done

    def idle(self) -> bool:
        return not self.active and not self.ready


# ---------------------------------------------------------------------------- GPU serving
@dataclasses.dataclass
class Built:
    rid: int
    problem: object
    op: object
    f: object
    u: object
    tol: float
    precision: str
    n_total: int
    build_ms: float


class _EngineAdapter:
    def __init__(self, engine, max_iter: int):
        self.e = engine
        self.max_iter = max_iter

    def submit(self, b: Built, tag: int) -> bool:
        return self.e.submit(b.op, b.f, b.u, b.tol, b.precision, self.max_iter, tag)

    def step(self, iters):
        return self.e.step(iters)

    def poll(self):
        return self.e.poll()


def serve(requests: Sequence, hbm_budget_bytes: int = 2 << 30, max_slots: int = 0, iters_per_tick: int = 4,
          build_threads: int = 2, ready_depth: int = 16, tol64: float = 1e-10, tol32: float = 1e-9,
          max_iter: int = 2000, keep_results: bool = False, realtime: bool = True, flags_for=None):
    """Serve ``requests`` (objects with ``d, a_freqs, a_hat, f_freqs, f_hat, level,
    precision, arrival_s``) on the current GPU.  Returns a summary dict and the
    list of ``Finished`` records (with ``result`` = host solution when
    ``keep_results``)."""
    import torch

    from . import sparsespec as ss

    dev = torch.device("cuda", torch.cuda.current_device())
    engine = ss.Engine(hbm_budget_bytes, max_slots)
    sched = Scheduler(_EngineAdapter(engine, max_iter), iters_per_tick)
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
    built_q: "queue.Queue[Built]" = queue.Queue()
    t0 = time.perf_counter()
    arrivals = [t0 + requests[i].arrival_s if realtime else t0 for i in range(len(requests))]
    next_job = [0]
    lock = threading.Lock()
    errors: List[BaseException] = []
    in_ready = threading.Semaphore(ready_depth)

    def builder():
        stream = torch.cuda.Stream(device=dev)
        while True:
            with lock:
                if next_job[0] >= len(order):
                    return
                i = order[next_job[0]]
                next_job[0] += 1
            wait = arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            in_ready.acquire()
            try:
                p = requests[i]
                tb = time.perf_counter()
                with torch.cuda.stream(stream):
                    st = ss.Stamp.build([p], stream=stream.cuda_stream)
                    flags = flags_for(p) if flags_for else 0
                    op = ss.Operator.build(st, [p], flags, stream=stream.cuda_stream)
                    f = st.forcing_vector([p], dev)
                    u = torch.zeros_like(f)
                    stream.synchronize()
                n_total = st.n_total
                st.close()
                tol = tol64 if p.precision == "fp64" else tol32
                built_q.put(Built(i, p, op, f, u, tol, p.precision, n_total, 1e3 * (time.perf_counter() - tb)))
            except BaseException as e:   # surfaced by the scheduler loop
                errors.append(e)
                in_ready.release()
                return

    threads = [threading.Thread(target=builder, daemon=True) for _ in range(build_threads)]
    for t in threads:
        t.start()
    n_done = 0
    build_ms = []
    ticks = 0
    results = {}

    def take(b: Built):
        sched.offer(b.rid, arrivals[b.rid], b)
        build_ms.append(b.build_ms)

    while n_done < len(requests):
        if errors:
            raise errors[0]
        moved = 0
        while True:
            try:
                take(built_q.get_nowait())
                moved += 1
            except queue.Empty:
                break
        for _ in range(sched.admit()):
            in_ready.release()          # bounded: built requests not yet admitted
        if sched.ready and not sched.active:
            raise RuntimeError("a request does not fit the engine's HBM budget even alone")
        if sched.active:
            before = len(sched.finished)
            sched.tick()
            ticks += 1
            for r in sched.finished[before:]:
                b: Built = r.result
                if keep_results:
                    results[r.rid] = b.u.cpu().numpy()
                b.op.close()            # frees the operator and its workspace
                r.result = None
            n_done = len(sched.finished)
        elif not moved:
            try:
                take(built_q.get(timeout=0.005))
            except queue.Empty:
                pass
    for t in threads:
        t.join()
    t_end = time.perf_counter()
    recs = sched.finished
    for r in recs:
        r.result = results.get(r.rid)
    lat = np.array([r.latency for r in recs]) * 1e3
    first = min(arrivals)
    summary = {
        "requests": len(recs),
        "solves_per_s": len(recs) / (t_end - first),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "max_active": sched.max_active,
        "ticks": ticks,
        "build_ms_mean": float(np.mean(build_ms)) if build_ms else 0.0,
        "status_ok": int(sum(1 for r in recs if r.info["status"] == 0)),
        "fp32_refine": int(sum(1 for i in range(len(requests)) if requests[i].precision != "fp64")),
        "hbm_budget_bytes": int(hbm_budget_bytes),
    }
    engine.close()
    recs.sort(key=lambda r: r.rid)
    return summary, recs
