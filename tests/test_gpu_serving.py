"""Serving loop on the GPU: every result is bitwise the same alone and in the
mix of overlapping, batched requests, and within the forward bar of the
oracle; the memory budget holds."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_00645_amd as dsk
from paper_2211_00645_amd import synth
from paper_2211_00645_amd.serving import GPUExecutor, Request, Scheduler, run_plain, summarize

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPES = [(64, 128), (128, 256)]      # (rows, cols) of the small test pool
MAXP = 60


@pytest.fixture(scope="module")
def pool():
    p = {}
    for k, (r, c) in enumerate(SHAPES):
        for ch in range(2):
            p[(r, c, ch)] = synth.blob_stack((MAXP, r, c), 40, 10 * k + ch, device=DEV)
    torch.cuda.synchronize()
    return p


def _trace(n, rate, seed):
    import numpy as np
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    t -= t[0]
    out = []
    for i in range(n):
        r, c = SHAPES[int(rng.integers(0, len(SHAPES)))]
        out.append(Request(rid=i, t_arrival=float(t[i]), planes=int(rng.integers(20, MAXP + 1)),
                           rows=r, cols=c, channels=2,
                           angle_deg=float(rng.choice([30.0, 35.0, 45.0]))))
    return out


def _check_alone(pool, reqs):
    for r in reqs:
        assert r.status == "done", r
        for ch in range(2):
            stack = pool[(r.rows, r.cols, ch)][:r.planes]
            solo = dsk.deskew(stack, r.angle_deg, r.step_um, r.pixel_um)
            torch.cuda.synchronize()
            got = r.result[ch]
            assert torch.equal(got["psum"], solo["psum"].cpu()), (r.rid, ch)
            assert torch.equal(got["pmax"], solo["pmax"].cpu()), (r.rid, ch)
            assert torch.equal(got["vol"], solo["vol"]), (r.rid, ch)


def _check_oracle(r, ch, stack_rows, rows, got, vol=None):
    """A served result against the oracle at the forward bar: projections
    (and the volume, when kept) within 1e-5 relative per element, padding
    voxels exactly zero.  ``stack_rows`` is the request's channel stack
    restricted to ``rows`` (rows are independent in the remap)."""
    sn = stack_rows.cpu().numpy()
    offs = oracle.offsets_uniform(sn.shape[0], oracle.shift_px(r.angle_deg, r.step_um,
                                                                r.pixel_um))
    ref = oracle.deskew(sn, offs, vol=vol is not None)
    assert ref["width"] == r.width, (r.rid, ch)
    r0, r1 = rows
    for k in ("psum", "pmax"):
        g = got[k][r0:r1].cpu().numpy().astype(np.float64)
        o = ref[k].astype(np.float64)
        assert (np.abs(g - o) <= 1e-5 * np.abs(o)).all(), (r.rid, ch, k)
    if vol is not None:
        g = vol[:, r0:r1].cpu().numpy().astype(np.float64)
        o = ref["vol"].astype(np.float64)
        assert (np.abs(g - o) <= 1e-5 * np.abs(o)).all(), (r.rid, ch, "vol")
        assert (g[o == 0] == 0).all(), (r.rid, ch)


def test_mixed_requests_equal_solo_runs(pool):
    reqs = _trace(24, 3000.0, 1)          # a burst: requests overlap on the GPU
    ex = GPUExecutor(pool, n_slots=3)
    ex.keep_results = True
    sch = Scheduler(ex, budget_bytes=1 << 34, n_slots=3, max_batch=4)
    done = sch.run(reqs)
    s = summarize(done)
    print(f"serving: {s} launches={sch.launches} max_inflight={sch.max_inflight}", flush=True)
    assert s["done"] == 24
    assert sch.launches < 24              # requests were batched
    _check_alone(pool, done)
    # and every served result against the oracle (whole stacks)
    for r in done:
        for ch in range(2):
            stack = pool[(r.rows, r.cols, ch)][:r.planes]
            _check_oracle(r, ch, stack, (0, r.rows), r.result[ch], vol=r.result[ch]["vol"])


def test_budget_holds_and_plain_baseline(pool):
    reqs = _trace(10, 5000.0, 2)
    ex = GPUExecutor(pool, n_slots=4)
    ex.keep_results = True
    from paper_2211_00645_amd.serving import request_bytes
    one = max(request_bytes(r, ex.width(r)) for r in reqs)
    sch = Scheduler(ex, budget_bytes=2 * one, n_slots=4, max_batch=8)
    done = sch.run(reqs)
    assert all(r.status == "done" for r in done)
    assert sch.peak_used <= sch.budget and sch.used == 0
    _check_alone(pool, done)
    plain = run_plain(GPUExecutor(pool, n_slots=1), _trace(10, 5000.0, 2))
    assert all(r.status == "done" for r in plain)


def test_arena_outputs_equal_solo_runs(pool):
    """Outputs placed in the executor's arena (here only about three
    requests large, so batches also wait for space): projections bitwise
    equal to solo runs."""
    from paper_2211_00645_amd.serving import request_bytes
    reqs = _trace(30, 4000.0, 3)
    probe = GPUExecutor(pool, n_slots=1)
    one = max(request_bytes(r, probe.width(r)) for r in reqs)
    ex = GPUExecutor(pool, n_slots=3, arena_bytes=3 * one)
    sch = Scheduler(ex, budget_bytes=3 * one, n_slots=3, max_batch=4)
    done = sch.run(reqs)
    print(f"arena: launches={sch.launches} space_waits={sch.space_waits}", flush=True)
    assert all(r.status == "done" for r in done)
    assert ex.arena.used == 0
    for r in done:
        for ch in range(2):
            solo = dsk.deskew(pool[(r.rows, r.cols, ch)][:r.planes], r.angle_deg, r.step_um,
                              r.pixel_um)
            torch.cuda.synchronize()
            assert torch.equal(r.result[ch]["psum"], solo["psum"].cpu()), (r.rid, ch)
            assert torch.equal(r.result[ch]["pmax"], solo["pmax"].cpu()), (r.rid, ch)


def test_failed_submit_returns_its_arena_block(pool):
    """A request the executor cannot serve (no stack of its shape in the
    pool) fails; its batch's arena block and budget are given back and the
    requests after it are served."""
    reqs = _trace(6, 2000.0, 4)
    reqs[2].rows, reqs[2].cols = 96, 128            # not in the pool
    ex = GPUExecutor(pool, n_slots=2, arena_bytes=1 << 30)
    sch = Scheduler(ex, budget_bytes=1 << 30, n_slots=2, max_batch=1)
    done = sch.run(reqs)
    status = {r.rid: r.status for r in done}
    assert status[2] == "failed"
    assert all(st == "done" for rid, st in status.items() if rid != 2)
    assert ex.arena.used == 0 and sch.used == 0


def test_full_size_burst_projections_equal_solo_runs():
    """The serving workload's sizes (2-channel stacks, 100-400 planes of
    512/1024 x 1024/2048): the first 16 requests of the benchmark's burst
    trace, batched through the scheduler with outputs in an arena, return
    projections bitwise equal to each channel's solo deskew."""
    from paper_2211_00645_amd import serving as sv
    big = {}
    for k, (r, c) in enumerate([(512, 1024), (512, 2048), (1024, 1024), (1024, 2048)]):
        for ch in range(2):
            big[(r, c, ch)] = synth.blob_stack((400, r, c), synth.blobs_for_volume(400, r, c),
                                               500 + 2 * k + ch, device=DEV)
    torch.cuda.synchronize()
    reqs = sv.make_requests(synth.serving_trace(16, 1e9, 7))
    ex = GPUExecutor(big, n_slots=4, arena_bytes=64 << 30)
    sch = Scheduler(ex, budget_bytes=64 << 30, n_slots=4, max_batch=8)
    done = sch.run(reqs)
    print(f"full-size burst: launches={sch.launches}", flush=True)
    assert all(r.status == "done" for r in done)
    assert ex.arena.used == 0
    for r in done:
        for ch in range(2):
            solo = dsk.deskew(big[(r.rows, r.cols, ch)][:r.planes], r.angle_deg, r.step_um,
                              r.pixel_um, vol=False)
            torch.cuda.synchronize()
            assert torch.equal(r.result[ch]["psum"], solo["psum"].cpu()), (r.rid, ch)
            assert torch.equal(r.result[ch]["pmax"], solo["pmax"].cpu()), (r.rid, ch)
            # sampled rows of the served projections against the oracle
            for r0 in (0, r.rows // 2 + 1, r.rows - 2):
                st = big[(r.rows, r.cols, ch)][:r.planes, r0:r0 + 2].contiguous()
                _check_oracle(r, ch, st, (r0, r0 + 2), r.result[ch])
    del big, ex
    torch.cuda.empty_cache()
