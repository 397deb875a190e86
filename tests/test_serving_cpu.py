"""Scheduler logic of the serving loop on the CPU, with a stand-in engine:
arrival-order admission, HBM-budget gating (never exceeded, refused requests
stay queued), retirement freeing capacity for later arrivals, per-request
accounting of multi-problem requests, and latency bookkeeping."""
import pytest

from paper_2302_00752_amd.serving import Scheduler


class FakeEngine:
    """Admits a request if its bytes fit the budget; each problem needs `steps` ticks."""

    def __init__(self, budget):
        self.budget = budget
        self.used = 0
        self.active = {}          # tag -> [bytes, remaining ticks, n_prob]
        self.out = []
        self.peak = 0
        self.admit_log = []

    def submit(self, handle, tag):
        if self.used + handle["bytes"] > self.budget:
            return False
        self.used += handle["bytes"]
        self.peak = max(self.peak, self.used)
        self.active[tag] = [handle["bytes"], handle["steps"], handle["n_prob"]]
        self.admit_log.append(tag)
        return True

    def step(self, iters):
        for tag in list(self.active):
            rec = self.active[tag]
            rec[1] -= 1
            if rec[1] <= 0:
                for p in range(rec[2]):
                    self.out.append((tag, p, {"status": 0}))
                self.used -= rec[0]
                del self.active[tag]
        return len(self.active)

    def poll(self):
        out, self.out = self.out, []
        return out


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def test_budget_gating_order_and_completion():
    eng = FakeEngine(budget=100)
    clock = Clock()
    s = Scheduler(eng, clock=clock)
    sizes = [40, 40, 40, 10, 90, 5]
    for i, b in enumerate(sizes):
        s.offer(i, 0.0, {"bytes": b, "steps": 2 + i % 3, "n_prob": 1})
    ticks = 0
    while not s.idle():
        s.admit()
        assert eng.used <= eng.budget
        clock.t += 1.0
        s.tick()
        ticks += 1
        assert ticks < 100
    assert eng.peak <= 100
    assert eng.admit_log == sorted(eng.admit_log)          # first come, first admitted
    assert sorted(r.rid for r in s.finished) == list(range(len(sizes)))
    assert s.max_active >= 2                                 # requests overlap on the device


def test_late_arrivals_join_running_batch():
    eng = FakeEngine(budget=1000)
    clock = Clock()
    s = Scheduler(eng, clock=clock)
    s.offer(0, 0.0, {"bytes": 10, "steps": 5, "n_prob": 1})
    s.admit()
    s.tick()
    clock.t = 1.0
    s.offer(1, 1.0, {"bytes": 10, "steps": 1, "n_prob": 1})   # arrives while 0 is running
    s.admit()
    assert set(s.active) == {0, 1}
    clock.t = 2.0
    s.tick()
    assert [r.rid for r in s.finished] == [1]                # the short late request finishes first
    assert s.finished[0].latency == pytest.approx(1.0)


def test_multi_problem_request_finishes_once():
    eng = FakeEngine(budget=1000)
    s = Scheduler(eng, clock=Clock())
    s.offer(7, 0.0, {"bytes": 1, "steps": 1, "n_prob": 3}, n_prob=3)
    s.admit()
    assert s.tick() == 1
    assert len(s.finished) == 1 and s.finished[0].rid == 7


def test_refused_request_stays_queued():
    eng = FakeEngine(budget=50)
    s = Scheduler(eng, clock=Clock())
    s.offer(0, 0.0, {"bytes": 40, "steps": 3, "n_prob": 1})
    s.offer(1, 0.0, {"bytes": 40, "steps": 1, "n_prob": 1})
    assert s.admit() == 1 and len(s.ready) == 1
    for _ in range(3):
        s.tick()
    assert s.admit() == 1 and not s.ready


def test_refusals_and_joins_are_counted():
    eng = FakeEngine(budget=50)
    s = Scheduler(eng, clock=Clock())
    s.offer(0, 0.0, {"bytes": 30, "steps": 3, "n_prob": 1})
    assert s.admit() == 1 and s.refusals == 0 and s.joined_running == 0
    s.tick()                                                   # 0 is now mid-solve
    s.offer(1, 1.0, {"bytes": 30, "steps": 1, "n_prob": 1})   # does not fit beside 0
    s.offer(2, 1.0, {"bytes": 10, "steps": 1, "n_prob": 1})
    assert s.admit() == 0 and s.refusals == 1                 # head of the queue refused, order kept
    s.tick()
    s.tick()                                                  # 0 retires
    assert s.admit() == 2 and s.joined_running == 0           # nothing was running any more
    s.offer(3, 2.0, {"bytes": 5, "steps": 3, "n_prob": 1})
    s.admit()
    s.tick()
    s.offer(4, 3.0, {"bytes": 5, "steps": 1, "n_prob": 1})
    s.admit()
    assert s.joined_running == 1                              # 4 joined 3, admitted a tick earlier
    while not s.idle():
        s.admit()
        s.tick()
    fin = {r.rid: r for r in s.finished}
    assert sorted(fin) == [0, 1, 2, 3, 4]
    assert fin[4].admit_tick > fin[3].admit_tick and fin[4].admit_tick < fin[3].done_tick


def test_serve_refuses_more_than_two_builders():
    from paper_2302_00752_amd.serving import serve
    with pytest.raises(ValueError):
        serve([], build_threads=4)


# ---------------------------------------------------------------- the request loop with stand-ins
import dataclasses
import random
import threading
import time

import numpy as np

from paper_2302_00752_amd.serving import serve_loop


@dataclasses.dataclass
class Req:
    d: int
    precision: str
    arrival_s: float
    rows: int


class BuiltEngine:
    """Stand-in engine for serve_loop: a build costs 10 bytes per request; its problems finish
    two ticks after admission."""

    def __init__(self, budget=10 ** 9):
        self.budget, self.used, self.active, self.out = budget, 0, {}, []
        self.lock = threading.Lock()   # the loop calls it from one thread; checked anyway

    def submit(self, b, tag):
        assert self.lock.acquire(blocking=False), "engine entered from two threads"
        try:
            n = len(b.rids)
            if self.used + 10 * n > self.budget:
                return False
            self.used += 10 * n
            self.active[tag] = [10 * n, 2, n]
            return True
        finally:
            self.lock.release()

    def step(self, iters):
        for tag in list(self.active):
            rec = self.active[tag]
            rec[1] -= 1
            if rec[1] <= 0:
                self.out += [(tag, p, {"status": 0}) for p in range(rec[2])]
                self.used -= rec[0]
                del self.active[tag]
        return len(self.active)

    def poll(self):
        out, self.out = self.out, []
        return out

    def usage(self):
        return len(self.active), self.used


def standin_build(delay=0.0, fail_at=None, block=None):
    """build(probs, flags) -> (op, f, u, offsets): u holds 1000 * rows + index for each problem's rows."""
    calls = [0]
    lock = threading.Lock()

    def build(probs, flags):
        with lock:
            calls[0] += 1
            k = calls[0]
        if fail_at is not None and k == fail_at:
            raise ValueError(f"stand-in build {k} failed")
        if block is not None:
            block.wait()
        if delay:
            time.sleep(random.uniform(0, delay))
        offs = np.cumsum([0] + [p.rows for p in probs])
        u = np.concatenate([1000 * p.rows + np.arange(p.rows) for p in probs])
        return object(), None, u, offs

    return build


def run_loop(reqs, build, eng=None, **kw):
    eng = eng or BuiltEngine()
    return serve_loop(reqs, eng, eng.usage, build, solution=lambda b, lo, hi: b.u[lo:hi].copy(),
                      release=lambda b: None, **kw)


@pytest.mark.timeout(60)
@pytest.mark.parametrize("threads", [1, 2, 4, 8])
def test_loop_with_many_builders_serves_every_request_once(threads):
    random.seed(threads)
    reqs = [Req(3, "fp64" if i % 3 else "fp32_refine", 0.0002 * i, 5 + i % 17) for i in range(300)]
    summary, recs = run_loop(reqs, standin_build(delay=0.002), eng=BuiltEngine(budget=400), build_threads=threads,
                             keep_results=True, max_group=8, stall_timeout_s=20)
    assert summary["requests"] == len(reqs) and [r.rid for r in recs] == list(range(len(reqs)))
    for r in recs:   # every request got its own rows back
        assert np.array_equal(r.result, 1000 * reqs[r.rid].rows + np.arange(reqs[r.rid].rows))
    assert summary["build_threads"] == threads


@pytest.mark.timeout(60)
def test_loop_build_error_ends_the_run():
    reqs = [Req(3, "fp64", 0.0, 4) for _ in range(50)]
    with pytest.raises(ValueError, match="stand-in build 3 failed"):
        run_loop(reqs, standin_build(fail_at=3), build_threads=4, max_group=2, realtime=False)


@pytest.mark.timeout(60)
def test_loop_error_while_grouping_ends_the_run():
    # an error before the build (here in the flags callback) ends the run instead of leaving the
    # taken requests unbuilt and the loop waiting for them
    reqs = [Req(3, "fp64", 0.0, 4) for _ in range(20)]

    def flags_for(p):
        if p is reqs[7]:
            raise KeyError("no flags for request 7")
        return 0

    with pytest.raises(KeyError, match="no flags"):
        run_loop(reqs, standin_build(), build_threads=4, max_group=1, realtime=False, flags_for=flags_for)


@pytest.mark.timeout(60)
def test_loop_stall_is_reported():
    block = threading.Event()
    reqs = [Req(3, "fp64", 0.0, 4) for _ in range(10)]
    try:
        with pytest.raises(RuntimeError, match="no progress .* builders: building"):
            run_loop(reqs, standin_build(block=block), build_threads=4, realtime=False, stall_timeout_s=0.5)
    finally:
        block.set()
