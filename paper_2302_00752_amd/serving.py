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
    prob: int = 0           # problem of the unit's handle that answered this request (grouped builds)
    admit_tick: int = 0     # ticks run before the request's unit was admitted
    done_tick: int = 0      # ticks run when it finished
    offered: float = 0.0    # when its built unit became ready for admission

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class _Unit:
    """What the engine admits in one submit: a handle whose problems answer one or more requests.
    ``reqs`` holds [rid, arrival, problems left]; with ``per_problem`` request i is problem i."""
    tag: int
    handle: object
    reqs: list
    n_prob: int
    per_problem: bool
    admitted: float = 0.0
    left: int = 0
    offered: float = 0.0
    admit_tick: int = 0


class Scheduler:
    """Admission and retirement bookkeeping for one engine.

    ``engine`` must provide ``submit(handle, tag) -> bool`` (False when the
    budget or slots are exhausted), ``step(iters) -> n_active`` and
    ``poll() -> [(tag, prob, info)]``.  ``handle`` is whatever the builder made;
    with ``offer`` it answers one request, finished when all ``n_prob`` of its
    problems have been polled; with ``offer_group`` (one build for several
    requests) problem i answers request i.  Handles whose problems are all done
    are listed in ``retired`` for the caller to release.
    """

    def __init__(self, engine, iters_per_tick: int = 4, clock: Callable[[], float] = time.perf_counter):
        self.engine = engine
        self.iters = iters_per_tick
        self.clock = clock
        self.ready: collections.deque = collections.deque()      # _Unit, in arrival order
        self.active: Dict[int, _Unit] = {}                         # tag -> unit
        self.finished: List[Finished] = []
        self.retired: List[object] = []
        self.max_active = 0
        self.ticks = 0              # engine steps run so far
        self.refusals = 0           # admission attempts the engine refused (budget or slots)
        self.joined_running = 0     # units admitted while a unit admitted at an earlier tick was active

    def offer(self, rid: int, arrival: float, handle, n_prob: int = 1):
        self.ready.append(_Unit(rid, handle, [[rid, arrival, n_prob]], n_prob, False, offered=self.clock()))

    def offer_group(self, tag: int, handle, reqs):
        """``reqs``: [(rid, arrival)] answered by problems 0, 1, ... of ``handle``."""
        self.ready.append(_Unit(tag, handle, [[rid, arr, 1] for rid, arr in reqs], len(reqs), True,
                                offered=self.clock()))

    def admit(self) -> int:
        """Admit ready units in arrival order until the engine refuses one."""
        n = 0
        while self.ready:
            u = self.ready[0]
            if not self.engine.submit(u.handle, u.tag):
                self.refusals += 1
                break
            self.ready.popleft()
            if any(a.admit_tick < self.ticks for a in self.active.values()):
                self.joined_running += 1
            u.admitted = self.clock()
            u.admit_tick = self.ticks
            u.left = u.n_prob
            self.active[u.tag] = u
            n += 1
        self.max_active = max(self.max_active, len(self.active))
        return n

    def tick(self) -> int:
        """One engine step plus retirement; returns the number of requests finished."""
        if not self.active:
            return 0
        self.engine.step(self.iters)
        self.ticks += 1
        done = 0
        for tag, prob, info in self.engine.poll():
            u = self.active[tag]
            req = u.reqs[prob] if u.per_problem else u.reqs[0]
            req[2] -= 1
            if req[2] == 0:
                self.finished.append(Finished(req[0], req[1], u.admitted, self.clock(), info, u.handle,
                                              prob if u.per_problem else 0, u.admit_tick, self.ticks,
                                              u.offered))
                done += 1
            u.left -= 1
            if u.left == 0:
                self.active.pop(tag)
                self.retired.append(u.handle)
        return done

    def idle(self) -> bool:
        return not self.active and not self.ready


# ---------------------------------------------------------------------------- GPU serving
@dataclasses.dataclass
class Built:
    """One build (stamps, operator, f, u) answering the requests ``rids``: problem i is request
    rids[i], its entries of f and u at [offsets[i], offsets[i+1])."""
    tag: int
    rids: list
    op: object
    f: object
    u: object
    offsets: object
    tol: float
    precision: str
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


def _padded(p, d: int):
    """The same problem on the d-torus, d >= p.d: every frequency gets zero coordinates appended.
    Its stamping set, operator and solution are those of p, keys padded alike (all dot products and
    norms are unchanged, and lexicographic order is kept)."""
    if p.d == d:
        return p
    q = dataclasses.replace(p)
    q.d = d
    q.a_freqs = np.pad(np.asarray(p.a_freqs), ((0, 0), (0, d - p.d)))
    q.f_freqs = np.pad(np.asarray(p.f_freqs), ((0, 0), (0, d - p.d)))
    return q


def serve(requests: Sequence, hbm_budget_bytes: int = 2 << 30, max_slots: int = 0, iters_per_tick: int = 4,
          build_threads: int = 2, ready_depth: int = 16, tol64: float = 1e-10, tol32: float = 1e-9,
          max_iter: int = 2000, keep_results: bool = False, realtime: bool = True, flags_for=None,
          max_group: int = 64, stall_timeout_s: float = 120.0):
    """Serve ``requests`` (objects with ``d, a_freqs, a_hat, f_freqs, f_hat, level,
    precision, arrival_s``) on the current GPU.  A builder takes the next request once it
    has arrived together with every later one already arrived (at most ``max_group``) and
    builds each precision's share as one batch, dimensions padded to the largest.  Returns
    a summary dict and the list of ``Finished`` records (with ``result`` = host solution
    when ``keep_results``).

    At most two builder threads are allowed: a run with four stopped making progress on the
    GPU host and its cause has not been found, so larger counts are refused rather than run.
    A run that makes no progress for ``stall_timeout_s`` seconds while no request is still to
    arrive raises, naming what every builder was doing."""
    if not 1 <= build_threads <= 2:
        raise ValueError("serve() runs one or two builder threads (a four-thread run stopped making "
                         "progress and its cause is not known)")
    import torch

    from . import sparsespec as ss

    dev = torch.device("cuda", torch.cuda.current_device())
    engine = ss.Engine(hbm_budget_bytes, max_slots)
    local = threading.local()

    def build(probs, flags):
        """Stamps, operator, f and u = 0 of one batch on this builder thread's own stream."""
        stream = getattr(local, "stream", None)
        if stream is None:
            stream = local.stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(stream):
            st = ss.Stamp.build(probs, stream=stream.cuda_stream)
            op = ss.Operator.build(st, probs, flags, stream=stream.cuda_stream)
            f = st.forcing_vector(probs, dev, stream=stream.cuda_stream)
            u = torch.zeros_like(f)
            stream.synchronize()
        offsets = st.offsets.copy()
        st.close()
        return op, f, u, offsets

    try:
        summary, recs = serve_loop(requests, _EngineAdapter(engine, max_iter), engine.usage, build,
                                   solution=lambda b, lo, hi: b.u[lo:hi].cpu().numpy(),
                                   release=lambda b: b.op.close(), iters_per_tick=iters_per_tick,
                                   build_threads=build_threads, ready_depth=ready_depth, tol64=tol64,
                                   tol32=tol32, keep_results=keep_results, realtime=realtime,
                                   flags_for=flags_for, max_group=max_group, stall_timeout_s=stall_timeout_s)
    finally:
        engine.close()
    summary["hbm_budget_bytes"] = int(hbm_budget_bytes)
    return summary, recs


def serve_loop(requests: Sequence, adapter, usage, build, solution, release, iters_per_tick: int = 4,
               build_threads: int = 2, ready_depth: int = 16, tol64: float = 1e-10, tol32: float = 1e-9,
               keep_results: bool = False, realtime: bool = True, flags_for=None, max_group: int = 64,
               stall_timeout_s: float = 120.0):
    """The request loop of ``serve`` over any engine and builder.

    ``adapter``: submit / step / poll as ``Scheduler`` expects them; ``usage() -> (slots,
    bytes)`` of the engine; ``build(probs, flags) -> (op, f, u, offsets)`` runs on a builder
    thread; ``solution(built, lo, hi)`` returns a host copy of u[lo:hi]; ``release(built)``
    frees a retired build.  Every builder's work, from taking requests to queueing the build,
    runs under one handler, so an error anywhere in it ends the run with that error; a run whose
    builders have all ended with requests unbuilt, or that makes no progress for
    ``stall_timeout_s`` seconds while no request is still to arrive, raises too."""
    sched = Scheduler(adapter, iters_per_tick)
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
    built_q: "queue.Queue[Built]" = queue.Queue()
    t0 = time.perf_counter()
    arrivals = [t0 + requests[i].arrival_s if realtime else t0 for i in range(len(requests))]
    next_job = [0]
    next_tag = [0]
    lock = threading.Lock()
    errors: List[BaseException] = []
    in_ready = threading.Semaphore(ready_depth)
    phase = ["starting"] * build_threads   # what every builder is doing (stall reports)

    def builder(w: int):
        try:
            while True:
                with lock:
                    if next_job[0] >= len(order):
                        phase[w] = "done"
                        return
                    first = order[next_job[0]]
                    next_job[0] += 1
                wait = arrivals[first] - time.perf_counter()
                if wait > 0:
                    phase[w] = f"waiting for request {first} to arrive"
                    time.sleep(wait)
                group = [first]
                with lock:   # every request that has arrived meanwhile joins the build
                    now = time.perf_counter()
                    while next_job[0] < len(order) and len(group) < max_group and arrivals[order[next_job[0]]] <= now:
                        group.append(order[next_job[0]])
                        next_job[0] += 1
                shares = collections.OrderedDict()
                for i in group:
                    p = requests[i]
                    shares.setdefault((p.precision, flags_for(p) if flags_for else 0), []).append(i)
                for (prec, flags), rids in shares.items():
                    phase[w] = f"waiting for a ready slot ({len(rids)} requests built next)"
                    in_ready.acquire()
                    phase[w] = f"building {len(rids)} requests from request {rids[0]}"
                    tb = time.perf_counter()
                    dmax = max(requests[i].d for i in rids)
                    probs = [_padded(requests[i], dmax) for i in rids]
                    op, f, u, offsets = build(probs, flags)
                    with lock:
                        tag = next_tag[0]
                        next_tag[0] += 1
                    tol = tol64 if prec == "fp64" else tol32
                    built_q.put(Built(tag, rids, op, f, u, offsets, tol, prec, 1e3 * (time.perf_counter() - tb)))
        except BaseException as e:   # surfaced by the scheduler loop
            phase[w] = f"failed: {e!r}"
            errors.append(e)
            in_ready.release()

    threads = [threading.Thread(target=builder, args=(w,), daemon=True) for w in range(build_threads)]
    for t in threads:
        t.start()
    n_done = 0
    n_built = 0
    build_ms = []
    group_sizes = []
    ticks = 0
    results = {}
    peak_bytes = 0
    max_unit = 0                        # largest footprint of a unit admitted on its own
    last_progress = time.perf_counter()

    def take(b: Built):
        nonlocal n_built
        sched.offer_group(b.tag, b, [(rid, arrivals[rid]) for rid in b.rids])
        build_ms.append(b.build_ms)
        group_sizes.append(len(b.rids))
        n_built += len(b.rids)

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
        before_bytes = usage()[1] if sched.ready else 0
        n_adm = sched.admit()
        for _ in range(n_adm):
            in_ready.release()          # bounded: built requests not yet admitted
        if n_adm:
            used = usage()[1]
            peak_bytes = max(peak_bytes, used)
            if n_adm == 1:
                max_unit = max(max_unit, used - before_bytes)
        if sched.ready and not sched.active:
            raise RuntimeError("the engine refused a request while it held no other")
        finished_before = n_done
        if sched.active:
            before = len(sched.finished)
            sched.tick()
            ticks += 1
            for r in sched.finished[before:]:
                b: Built = r.result
                if keep_results:
                    results[r.rid] = solution(b, int(b.offsets[r.prob]), int(b.offsets[r.prob + 1]))
                r.result = None
            for b in sched.retired:
                release(b)              # frees the operator and its workspace
            sched.retired.clear()
            n_done = len(sched.finished)
        elif not moved:
            try:
                take(built_q.get(timeout=0.005))
                moved += 1
            except queue.Empty:
                pass
        now = time.perf_counter()
        if moved or n_adm or n_done > finished_before:
            last_progress = now
        elif not sched.active and built_q.empty() and not any(t.is_alive() for t in threads):
            if errors:
                raise errors[0]
            raise RuntimeError(f"the builders ended with {len(requests) - n_built} requests unbuilt")
        elif not sched.active and now - last_progress > stall_timeout_s and \
                not any(ph.startswith("waiting for request") for ph in phase):
            raise RuntimeError(f"serving made no progress for {now - last_progress:.0f} s with "
                               f"{len(requests) - n_built} requests unbuilt, {len(sched.ready)} built units "
                               f"waiting; builders: " + "; ".join(phase))
    for t in threads:
        t.join()
    t_end = time.perf_counter()
    recs = sched.finished
    for r in recs:
        r.result = results.get(r.rid)
    lat = np.array([r.latency for r in recs]) * 1e3
    queued = np.array([r.admitted - r.offered for r in recs]) * 1e3     # built, waiting for admission
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
        "requests_per_build_mean": float(np.mean(group_sizes)) if group_sizes else 0.0,
        "status_ok": int(sum(1 for r in recs if r.info["status"] == 0)),
        "fp32_refine": int(sum(1 for i in range(len(requests)) if requests[i].precision != "fp64")),
        "peak_bytes_admitted": int(peak_bytes),
        "max_unit_bytes": int(max_unit),
        "refused_admissions": int(sched.refusals),
        "joined_running": int(sched.joined_running),
        "queue_ms_p50": float(np.percentile(queued, 50)),
        "queue_ms_p99": float(np.percentile(queued, 99)),
        "build_threads": int(build_threads),
    }
    recs.sort(key=lambda r: r.rid)
    return summary, recs
