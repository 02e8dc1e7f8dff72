"""Live serving loop: camera stacks arrive over time and are deskewed and
projected on the GPU under a device-memory budget.

The paper runs acquisition, processing and display as concurrent processes
so that a new stack can be acquired while the previous one is processed,
and lag grows without bound once processing is slower than acquisition
(methods section, Supp. Fig. 1).  The scheduler here is the GPU side of that
pipeline, with continuous batching:

  * requests (one multi-channel stack each) arrive with timestamps;
  * a request is admitted when a launch slot (a stream) is free and its
    bytes (input + volume + projections) fit in the remaining budget;
    requests larger than the whole budget are rejected;
  * all admitted requests waiting at that moment go out together in ONE
    persistent launch over every channel of every request, so work that
    arrives while other work is on the GPU joins as soon as a slot frees;
  * completion is an event after the projections' copy to host; it frees
    the slot and the request's bytes, which admits waiting requests.

The scheduler is plain host logic driven by a clock and an executor, so it
is tested on the CPU with a fake clock and a mock executor.
"""
from __future__ import annotations

import contextlib
import gc
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np

from .arena import Arena, NoSpace


@dataclass
class Request:
    rid: int
    t_arrival: float
    planes: int
    rows: int
    cols: int
    channels: int = 2
    angle_deg: float = 35.0
    step_um: float = 0.4
    pixel_um: float = 0.115
    nbytes: int = 0
    width: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    status: str = "new"            # queued / running / done / rejected / failed
    result: Any = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def out_voxels(self) -> int:
        return self.channels * self.planes * self.rows * self.width


def request_bytes(req: Request, width: int, keep_volume: bool = True) -> int:
    """Device bytes a request holds while in flight: the uint16 input, the
    float32 volume (if produced) and the two float32 projections, per
    channel."""
    per = 2 * req.planes * req.rows * req.cols + 8 * req.rows * width
    if keep_volume:
        per += 4 * req.planes * req.rows * width
    return req.channels * per


class RealClock:
    """Wall time in seconds since the clock was started (request arrival
    times are relative to that origin)."""

    def __init__(self):
        self.t0 = time.perf_counter()

    def start(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def idle(self, until: Optional[float]):
        dt = 1e-4 if until is None else min(1e-4, max(0.0, until - self.now()))
        if dt > 0:
            time.sleep(dt)


class FakeClock:
    """Virtual time: idle() jumps to the next event."""

    def __init__(self):
        self.t = 0.0

    def start(self):
        pass

    def now(self) -> float:
        return self.t

    def idle(self, until: Optional[float]):
        if until is None:
            raise RuntimeError("fake clock idle with no pending event")
        self.t = max(self.t, until)


class Scheduler:
    """Admission by memory budget, launch slots, continuous batching."""

    def __init__(self, executor, budget_bytes: int, n_slots: int = 4, max_batch: int = 8,
                 clock=None, keep_volume: bool = True, on_complete=None):
        if n_slots < 1 or max_batch < 1:
            raise ValueError("need at least one slot and one request per batch")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.n_slots = n_slots
        self.max_batch = max_batch
        self.clock = clock or RealClock()
        self.keep_volume = keep_volume
        # called with each request as it completes (a live display draws its
        # projections here and lets them go)
        self.on_complete = on_complete
        self.used = 0
        self.peak_used = 0
        self.launches = 0
        self.max_inflight = 0
        self.space_waits = 0

    def run(self, requests: List[Request]) -> List[Request]:
        """Serve ``requests`` (arrival times relative to the start of the
        run: the clock starts once the loop is about to begin, after the
        garbage-collector pause's collection)."""
        with gc_paused():
            self.clock.start()
            return self._run(requests)

    def _run(self, requests: List[Request]) -> List[Request]:
        arrivals = sorted(requests, key=lambda r: r.t_arrival)
        for r in arrivals:
            r.width = self.ex.width(r)
            r.nbytes = request_bytes(r, r.width, self.keep_volume)
        ai = 0
        queue: deque = deque()
        inflight: Dict[int, Any] = {}
        free = list(range(self.n_slots))[::-1]
        done: List[Request] = []
        while ai < len(arrivals) or queue or inflight:
            progressed = False
            now = self.clock.now()
            while ai < len(arrivals) and arrivals[ai].t_arrival <= now:
                r = arrivals[ai]
                ai += 1
                if r.nbytes > self.budget:
                    r.status = "rejected"
                    r.t_done = now
                    done.append(r)
                else:
                    r.status = "queued"
                    queue.append(r)
                progressed = True
            for slot in list(inflight):
                tok, rs = inflight[slot]
                if self.ex.done(tok):
                    ok = self.ex.finish(tok)
                    t = self.clock.now()
                    for r in rs:
                        r.t_done = t
                        r.status = "done" if ok else "failed"
                        self.used -= r.nbytes
                        done.append(r)
                    if self.on_complete is not None:
                        for r in rs:
                            self.on_complete(r)
                    del inflight[slot]
                    free.append(slot)
                    progressed = True
            while free and queue:
                batch, nb = [], 0
                while (queue and len(batch) < self.max_batch
                       and self.used + nb + queue[0].nbytes <= self.budget):
                    r = queue.popleft()
                    batch.append(r)
                    nb += r.nbytes
                if not batch:
                    break                      # head of line waits for memory
                slot = free.pop()
                self.used += nb
                self.peak_used = max(self.peak_used, self.used)
                t = self.clock.now()
                for r in batch:
                    r.t_admit = t
                    r.status = "running"
                try:
                    tok = self.ex.submit(slot, batch)
                except NoSpace:
                    # the executor's memory is fragmented: the batch goes back
                    # to the head of the queue until a completion frees space
                    for r in reversed(batch):
                        r.status = "queued"
                        r.t_admit = math.nan
                        queue.appendleft(r)
                    self.used -= nb
                    free.append(slot)
                    self.space_waits += 1
                    if not inflight:
                        raise RuntimeError("executor has no space with nothing in flight")
                    break
                except Exception:
                    for r in batch:
                        r.status = "failed"
                        r.t_done = self.clock.now()
                        self.used -= r.nbytes
                        done.append(r)
                    free.append(slot)
                    continue
                inflight[slot] = (tok, batch)
                self.launches += 1
                self.max_inflight = max(self.max_inflight, len(inflight))
                progressed = True
            if not progressed:
                nxt = arrivals[ai].t_arrival if ai < len(arrivals) else None
                nc = self.ex.next_completion() if inflight else None
                cands = [t for t in (nxt, nc) if t is not None]
                self.clock.idle(min(cands) if cands else None)
        return done


@contextlib.contextmanager
def gc_paused():
    """Pause Python's cyclic garbage collector for a serving loop (reference
    counting still frees every request's objects at once): a collection
    pass over a large heap can stall the loop for tens of milliseconds and
    land inside a request's latency.  One collection runs before the loop
    starts; the previous setting is restored, and one collection runs, on
    exit."""
    was = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()
            gc.collect()


def run_plain(executor, requests: List[Request], clock=None, on_complete=None) -> List[Request]:
    """Baseline: one stack at a time in arrival order, each waited for
    before the next starts (no overlap, no batching).  ``on_complete`` as
    for :class:`Scheduler`."""
    with gc_paused():
        return _run_plain(executor, requests, clock, on_complete)


def _run_plain(executor, requests: List[Request], clock=None, on_complete=None) -> List[Request]:
    clock = clock or RealClock()
    clock.start()
    out = []
    for r in sorted(requests, key=lambda q: q.t_arrival):
        r.width = executor.width(r)
        r.nbytes = request_bytes(r, r.width)
        while clock.now() < r.t_arrival:
            clock.idle(r.t_arrival)
        r.t_admit = clock.now()
        tok = executor.submit(0, [r])
        while not executor.done(tok):
            clock.idle(executor.next_completion())
        ok = executor.finish(tok)
        r.t_done = clock.now()
        r.status = "done" if ok else "failed"
        out.append(r)
        if on_complete is not None:
            on_complete(r)
    return out


def summarize(done: List[Request]) -> dict:
    ok = [r for r in done if r.status == "done"]
    lat = np.array([r.latency for r in ok]) if ok else np.array([math.nan])
    t0 = min(r.t_arrival for r in done) if done else 0.0
    t1 = max(r.t_done for r in ok) if ok else 0.0
    span = max(t1 - t0, 1e-12)
    vox = sum(r.out_voxels for r in ok)
    return {
        "requests": len(done),
        "done": len(ok),
        "rejected": sum(r.status == "rejected" for r in done),
        "failed": sum(r.status == "failed" for r in done),
        "stacks_per_s": len(ok) / span,
        "voxels_per_s": vox / span,
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
        "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "latency_max_ms": float(np.max(lat) * 1e3),
        "span_s": span,
    }


def make_requests(trace, angle_deg=35.0, step_um=0.4, pixel_um=0.115) -> List[Request]:
    """Requests from ``synth.serving_trace`` records."""
    return [Request(rid=i, t_arrival=t["t"], planes=t["planes"], rows=t["rows"],
                    cols=t["cols"], channels=t["channels"], angle_deg=angle_deg,
                    step_um=step_um, pixel_um=pixel_um) for i, t in enumerate(trace)]


# --------------------------------------------------------------- executors

class MockExecutor:
    """CPU stand-in: a request batch takes ``s_per_byte`` * bytes of virtual
    time after the later of its submission and the previous completion on
    the same slot; ``fail_rids`` makes the batch holding those requests
    report failure."""

    def __init__(self, clock: FakeClock, s_per_byte: float = 1e-10, width_fn=None,
                 fail_rids=(), arena_bytes=None):
        self.clock = clock
        self.s_per_byte = s_per_byte
        self.width_fn = width_fn or (lambda r: r.cols + r.planes)
        self.fail = set(fail_rids)
        self.pending: Dict[int, tuple] = {}
        self.k = 0
        self.submitted: List[List[int]] = []
        self.arena = Arena(arena_bytes, align=1) if arena_bytes else None

    def width(self, r):
        return self.width_fn(r)

    def submit(self, slot, reqs):
        nb = sum(r.nbytes for r in reqs)
        off = self.arena.alloc(nb) if self.arena else None
        t_end = self.clock.now() + nb * self.s_per_byte
        self.k += 1
        self.pending[self.k] = (t_end, [r.rid for r in reqs], off)
        self.submitted.append([r.rid for r in reqs])
        return self.k

    def done(self, tok):
        return self.clock.now() >= self.pending[tok][0]

    def next_completion(self):
        return min(v[0] for v in self.pending.values()) if self.pending else None

    def finish(self, tok):
        _, rids, off = self.pending.pop(tok)
        if off is not None:
            self.arena.free(off)
        return not (set(rids) & self.fail)


class GPUExecutor:
    """Deskew + projections on the GPU.  Inputs come from a device-resident
    pool (``pool[(rows, cols, channel)]`` is a uint16 [max_planes][rows]
    [cols] tensor; a request uses its first ``planes`` planes), standing in
    for camera frames already delivered to HBM.  Each submit is ONE
    persistent launch over all channels of all requests in the batch on the
    slot's stream, followed by the projections' copy to a pinned host
    buffer of the batch and an event; each request's results are views of
    that buffer (it is freed, back to the pinned-memory cache, when they
    are).

    Outputs live in one device arena of ``arena_bytes`` reserved up front
    (first fit, freed at completion; :class:`NoSpace` when fragmented), so
    the loop never allocates device memory per request.  With
    ``keep_results`` the outputs are allocated separately instead and kept
    with the request (for checking)."""

    def __init__(self, pool, n_slots=4, tune=None, keep_volume=True, max_jobs=64,
                 arena_bytes=8 << 30):
        import torch
        from .batch import JobLauncher
        self.torch = torch
        self.pool = pool
        self.tune = tune
        self.keep_volume = keep_volume
        dev = next(iter(pool.values())).device
        self.device = dev
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_slots)]
        self.launcher = JobLauncher(max_jobs=max_jobs, slots=2 * n_slots)
        self.keep_results = False
        self.arena = Arena(arena_bytes, align=256)
        self.buf = None                            # reserved on first use


    def width(self, r):
        from . import api
        return api.plan((r.planes, r.rows, r.cols),
                        shift=api.shift_px(r.angle_deg, r.step_um, r.pixel_um))[0]

    def _outputs(self, reqs):
        """(request, channel, n, rows, width) per job and the arena bytes."""
        items, total = [], 0
        for r in reqs:
            w = self.width(r)
            for ch in range(r.channels):
                items.append((r, ch, r.planes, r.rows, w))
                nb = 8 * r.rows * w + (4 * r.planes * r.rows * w if self.keep_volume else 0)
                total += self.arena.round(nb)
        return items, total

    def _view(self, base, off, shape):
        n = 1
        for v in shape:
            n *= v
        return self.buf[base + off: base + off + 4 * n].view(self.torch.float32).view(shape)

    def submit(self, slot, reqs):
        from .batch import plan_job
        torch = self.torch
        s = self.streams[slot]
        items, total = self._outputs(reqs)
        base = None
        if not self.keep_results:
            if self.buf is None:
                self.buf = torch.empty((self.arena.size,), dtype=torch.uint8, device=self.device)
            base = self.arena.alloc(total)        # raises NoSpace when fragmented
        launched = False
        try:
            # the batch's projections go to one pinned host buffer of its own,
            # from the framework's caching pinned allocator; the requests'
            # results are views of it, so it lives while they do and then
            # returns to the cache (reused only after the copies into it
            # have completed) -- no copy out and no fresh pageable memory
            # per request
            proj = sum(2 * rows * w for (_, _, _, rows, w) in items)
            st = torch.empty((max(proj, 1),), dtype=torch.float32, pin_memory=True)
            jobs, outs, host = [], [], []
            off = 0
            hoff = 0
            with torch.cuda.stream(s):
                for (r, ch, n, rows, w) in items:
                    stack = self.pool[(r.rows, r.cols, ch)][:r.planes]
                    out = None
                    if base is not None:
                        out = {"psum": self._view(base, off, (rows, w)),
                               "pmax": self._view(base, off + 4 * rows * w, (rows, w))}
                        nb = 8 * rows * w
                        if self.keep_volume:
                            out["vol"] = self._view(base, off + nb, (n, rows, w))
                            nb += 4 * n * rows * w
                        off += self.arena.round(nb)
                    job, res = plan_job(stack, r.angle_deg, r.step_um, r.pixel_um,
                                        vol=self.keep_volume, out=out)
                    jobs.append(job)
                    outs.append((r, ch, res))
                self.launcher.launch(jobs, self.tune, stream=s)
                launched = True
                for r, ch, res in outs:
                    m = res["psum"].numel()
                    hp = st[hoff: hoff + m].view(res["psum"].shape)
                    hm = st[hoff + m: hoff + 2 * m].view(res["pmax"].shape)
                    hoff += 2 * m
                    hp.copy_(res["psum"], non_blocking=True)
                    hm.copy_(res["pmax"], non_blocking=True)
                    host.append((hp, hm))
                ev = torch.cuda.Event()
                ev.record(s)
        except BaseException:
            # give the outputs' arena block back; once the launch is queued,
            # only after the stream has finished with it
            if base is not None:
                if launched:
                    s.synchronize()
                self.arena.free(base)
            raise
        return (ev, outs, host, base)

    def done(self, tok):
        return tok[0].query()

    def next_completion(self):
        return None

    def finish(self, tok):
        ev, outs, host, base = tok
        ev.synchronize()
        for (r, ch, res), (hp, hm) in zip(outs, host):
            if r.result is None:
                r.result = {}
            keep = {"psum": hp, "pmax": hm}
            if self.keep_results and "vol" in res:
                keep["vol"] = res["vol"]
            r.result[ch] = keep
        if base is not None:
            self.arena.free(base)
        return True
