"""Host logic of the serving loop, on a fake clock with a mock executor:
admission by memory budget, continuous batching, backpressure, rejection
and failure handling.  No GPU."""
import math

import pytest

from paper_2211_00645_amd import synth
from paper_2211_00645_amd.serving import (FakeClock, MockExecutor, Request, Scheduler,
                                          make_requests, request_bytes, run_plain, summarize)


def _reqs(times, planes=100, rows=64, cols=64, channels=2):
    return [Request(rid=i, t_arrival=t, planes=planes, rows=rows, cols=cols,
                    channels=channels) for i, t in enumerate(times)]


def _one_bytes(planes=100, rows=64, cols=64, channels=2):
    r = Request(0, 0.0, planes, rows, cols, channels)
    return request_bytes(r, cols + planes)


def test_request_bytes():
    r = Request(0, 0.0, 10, 4, 8, channels=2)
    assert request_bytes(r, 20) == 2 * (2 * 10 * 4 * 8 + 4 * 10 * 4 * 20 + 8 * 4 * 20)
    assert request_bytes(r, 20, keep_volume=False) == 2 * (2 * 10 * 4 * 8 + 8 * 4 * 20)


def test_all_complete_in_order_with_latency_at_least_service():
    clk = FakeClock()
    ex = MockExecutor(clk, s_per_byte=1e-9)
    reqs = _reqs([0.0, 0.01, 0.02, 0.5])
    done = Scheduler(ex, budget_bytes=10**12, n_slots=2, clock=clk).run(reqs)
    assert [r.status for r in done] == ["done"] * 4
    svc = reqs[0].nbytes * 1e-9
    for r in done:
        assert r.latency >= svc - 1e-12
        assert r.t_admit >= r.t_arrival
    s = summarize(done)
    assert s["done"] == 4 and s["latency_p99_ms"] >= s["latency_p50_ms"]


def test_burst_is_batched_continuously():
    clk = FakeClock()
    ex = MockExecutor(clk, s_per_byte=1e-9)
    # 10 arrive at once, 3 more while the first batch runs
    times = [0.0] * 10 + [0.001, 0.002, 0.003]
    sch = Scheduler(ex, budget_bytes=10**12, n_slots=1, max_batch=4, clock=clk)
    done = sch.run(_reqs(times))
    assert all(r.status == "done" for r in done)
    assert [len(b) for b in ex.submitted][:3] == [4, 4, 4]
    assert sum(len(b) for b in ex.submitted) == 13
    # FIFO: batches take requests in arrival order
    flat = [rid for b in ex.submitted for rid in b]
    assert flat == sorted(flat)


def test_budget_backpressure_never_exceeded():
    clk = FakeClock()
    ex = MockExecutor(clk, s_per_byte=1e-9)
    one = _one_bytes()
    sch = Scheduler(ex, budget_bytes=int(2.5 * one), n_slots=4, max_batch=8, clock=clk)
    reqs = _reqs([0.0] * 7)
    done = sch.run(reqs)
    assert all(r.status == "done" for r in done)
    assert sch.peak_used <= sch.budget
    assert max(len(b) for b in ex.submitted) <= 2
    assert sch.used == 0
    # later requests waited for memory
    assert max(r.t_admit - r.t_arrival for r in done) > 0


def test_oversize_request_rejected_others_served():
    clk = FakeClock()
    ex = MockExecutor(clk)
    one = _one_bytes()
    reqs = _reqs([0.0, 0.0, 0.0])
    reqs[1].planes = 10000
    done = Scheduler(ex, budget_bytes=3 * one, n_slots=2, clock=clk).run(reqs)
    st = {r.rid: r.status for r in done}
    assert st == {0: "done", 1: "rejected", 2: "done"}


def test_executor_failure_releases_slot_and_budget():
    clk = FakeClock()
    ex = MockExecutor(clk, s_per_byte=1e-9, fail_rids={2})
    sch = Scheduler(ex, budget_bytes=10**12, n_slots=1, max_batch=1, clock=clk)
    done = sch.run(_reqs([0.0, 0.0, 0.0, 0.0]))
    st = {r.rid: r.status for r in done}
    assert st[2] == "failed" and [st[i] for i in (0, 1, 3)] == ["done"] * 3
    assert sch.used == 0


def test_submit_exception_marks_batch_failed():
    clk = FakeClock()

    class Boom(MockExecutor):
        def submit(self, slot, reqs):
            if any(r.rid == 1 for r in reqs):
                raise RuntimeError("launch failed")
            return super().submit(slot, reqs)

    ex = Boom(clk, s_per_byte=1e-9)
    sch = Scheduler(ex, budget_bytes=10**12, n_slots=2, max_batch=1, clock=clk)
    done = sch.run(_reqs([0.0, 0.0, 0.0]))
    st = {r.rid: r.status for r in done}
    assert st == {0: "done", 1: "failed", 2: "done"}
    assert sch.used == 0


def test_overlap_beats_one_at_a_time_under_burst():
    times = [0.0] * 8
    clk = FakeClock()
    done_p = run_plain(MockExecutor(clk, s_per_byte=1e-9), _reqs(times), clock=clk)
    clk2 = FakeClock()
    done_s = Scheduler(MockExecutor(clk2, s_per_byte=1e-9), budget_bytes=10**12, n_slots=4,
                       max_batch=1, clock=clk2).run(_reqs(times))
    assert summarize(done_s)["latency_p99_ms"] < summarize(done_p)["latency_p99_ms"]


def test_make_requests_from_trace():
    tr = synth.serving_trace(50, 20.0, 5)
    reqs = make_requests(tr)
    assert len(reqs) == 50 and all(r.channels == 2 for r in reqs)
    assert all(100 <= r.planes <= 400 and r.rows in (512, 1024) and r.cols in (1024, 2048)
               for r in reqs)
    ts = [r.t_arrival for r in reqs]
    assert ts == sorted(ts) and ts[0] == 0.0
    mean_gap = (ts[-1] - ts[0]) / 49
    assert 0.02 < mean_gap < 0.1          # Poisson at 20 Hz
    assert not math.isnan(reqs[0].t_arrival)


def test_fragmented_executor_memory_requeues_batch():
    """The executor places outputs in an arena as large as the budget; when
    a batch fits the budget but no contiguous block, it goes back to the
    head of the queue and runs once a completion frees space."""
    import random
    rnd = random.Random(5)
    clk = FakeClock()
    reqs = [Request(rid=i, t_arrival=0.0005 * i, planes=rnd.choice([20, 60, 140]), rows=64,
                    cols=64, channels=2) for i in range(80)]
    big = max(request_bytes(r, r.cols + r.planes) for r in reqs)
    budget = 3 * big
    ex = MockExecutor(clk, s_per_byte=1e-9, arena_bytes=budget)
    sch = Scheduler(ex, budget_bytes=budget, n_slots=4, max_batch=2, clock=clk)
    done = sch.run(reqs)
    assert all(r.status == "done" for r in done) and len(done) == 80
    assert sch.space_waits > 0
    assert sch.peak_used <= budget and sch.used == 0
    assert ex.arena.used == 0
    # FIFO order of admission is kept across the requeues
    flat = [rid for b in ex.submitted for rid in b]
    assert sorted(set(flat)) == list(range(80))


def test_scheduler_pauses_and_restores_the_cyclic_collector():
    import gc
    seen = []

    class Probe(MockExecutor):
        def submit(self, slot, reqs):
            seen.append(gc.isenabled())
            return super().submit(slot, reqs)

    clock = FakeClock()
    ex = Probe(clock, s_per_byte=1e-9)
    was = gc.isenabled()
    done = Scheduler(ex, budget_bytes=1 << 40, n_slots=2, clock=clock).run(
        _reqs([0.0, 0.01, 0.02, 0.03]))
    assert [r.status for r in done] == ["done"] * 4
    assert seen and not any(seen)
    assert gc.isenabled() == was


def test_on_complete_sees_every_request_once_after_it_is_done():
    seen = []

    def hook(r):
        assert r.status == "done" and r.t_done >= r.t_arrival
        seen.append(r.rid)

    clk = FakeClock()
    ex = MockExecutor(clk, s_per_byte=1e-9)
    Scheduler(ex, budget_bytes=10**12, n_slots=2, clock=clk, on_complete=hook).run(
        _reqs([0.0, 0.001, 0.002, 0.5]))
    assert sorted(seen) == [0, 1, 2, 3]
    seen.clear()
    clk2 = FakeClock()
    run_plain(MockExecutor(clk2, s_per_byte=1e-9), _reqs([0.0, 0.1]), clock=clk2,
              on_complete=hook)
    assert seen == [0, 1]


def test_clock_starts_when_the_loop_starts():
    """Arrival times count from the start of the run itself, not from the
    scheduler's construction or the collector pause before the loop."""
    import time
    from paper_2211_00645_amd.serving import RealClock

    class Clk(FakeClock):
        def __init__(self):
            super().__init__()
            self.started = 0
            self.read_before_start = False

        def start(self):
            self.started += 1

        def now(self):
            if not self.started:
                self.read_before_start = True
            return super().now()

    clk = Clk()
    Scheduler(MockExecutor(clk), budget_bytes=10**12, clock=clk).run(_reqs([0.0, 0.1]))
    assert clk.started == 1 and not clk.read_before_start
    clk2 = Clk()
    run_plain(MockExecutor(clk2), _reqs([0.0, 0.1]), clock=clk2)
    assert clk2.started == 1 and not clk2.read_before_start
    rc = RealClock()
    time.sleep(0.03)
    rc.start()
    assert rc.now() < 0.02
