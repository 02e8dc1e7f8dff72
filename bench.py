#!/usr/bin/env python3
"""Benchmark of the deskew hot path on one MI355X.

Workload: one 512 x 512 x 2048 uint16 light-sheet stack (sheet angle 35 deg,
scan step 0.4 um, 115 nm pixels; synthetic Poisson background + 2000
Gaussian spots) already resident in HBM.  One step = geometry plan (Eq. 1,
host FP64) + one fused kernel writing the FP32 deskewed volume and its sum and
maximum projections.  Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, R, C = 512, 512, 2048
ANGLE, STEP, PIXEL = 35.0, 0.4, 0.115
SEED, BLOBS = 2, 2000
HBM_PEAK_GBS = 8000.0
METRIC = "deskewed voxels/s & HBM GB/s, 512×512×2048 u16 stack; p99 live-stack latency"
KERNEL_SOURCES = ["paper_2211_00645_amd/csrc/kernels.hpp",
                  "paper_2211_00645_amd/csrc/deskew.hip",
                  "paper_2211_00645_amd/csrc/common.hpp"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "forward_512x512x2048_pmc.md")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(summary=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary (the
    forward's by default), if it was taken on the kernel as it stands (else
    None)."""
    summary = summary or PMC_SUMMARY
    if not os.path.exists(summary):
        return None
    vals = {}
    with open(summary) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    try:
        return int(float(vals["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(n, r, c, w):
    # read the uint16 stack once, write the dense FP32 volume, write 2 projections
    return 2 * n * r * c + 4 * n * r * w + 8 * r * w


def cpu_baseline(stack_host, target_s):
    """The FP64 oracle timed on the host cores over a bounded sample of the
    same workload: whole-row slabs (all planes) grown until one pass takes
    about ``target_s``; if the full stack is faster than that, it is run
    repeatedly and the repeats are counted."""
    import oracle
    offs = oracle.offsets_uniform(N, oracle.shift_px(ANGLE, STEP, PIXEL))
    b, w = oracle.frame(offs, C)
    t0 = time.perf_counter()
    oracle.deskew(stack_host, offs, rows=(0, 4))
    dt = time.perf_counter() - t0
    rows = int(max(4, min(R, round(4 * target_s / max(dt, 1e-6)))))
    reps = 1
    if rows == R:
        t0 = time.perf_counter()
        oracle.deskew(stack_host, offs)
        one = time.perf_counter() - t0
        reps = int(max(1, min(200, math.ceil(target_s / max(one, 1e-6)))))
    log(f"cpu baseline: oracle on rows 0..{rows} x {reps} ({oracle.threads()} threads)")
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.deskew(stack_host, offs, rows=(0, rows))
    dt = time.perf_counter() - t0
    vox = N * rows * w * reps
    what = (f"rows 0..{rows} of" if rows < R else f"{reps} passes over") + \
        f" the {N}x{R}x{C} stack (all {N} planes, W={w})"
    res = {"value": vox / dt, "unit": "voxels/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{what}, FP64 volume + sum + max projections, {dt:.2f} s",
           "seconds": dt}
    # the same on one core, over fewer rows (about a tenth of the time)
    nt = oracle.threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.deskew(stack_host, offs, rows=(0, 1))
        one_row = time.perf_counter() - t0
        rows1 = int(max(1, min(R, round(0.1 * target_s / max(one_row, 1e-6)))))
        t0 = time.perf_counter()
        oracle.deskew(stack_host, offs, rows=(0, rows1))
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(nt)
    res["value_1core"] = N * rows1 * w / dt1
    res["sample_1core"] = f"rows 0..{rows1} on 1 thread, {dt1:.2f} s"
    res["host_cpus"] = os.cpu_count()
    res["cpu_model"] = _cpu_model()
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def config1_times(torch, dsk, synth):
    """The small stack (64 x 128 x 256 uint16, 30 deg, 0.4 um, 0.115 um; 50
    spots, seed 0): GPU forward (calls back to back) and the FP64 oracle on
    the host cores, median of 3.  Correctness-sized: it fits in the on-die
    cache, so it says nothing about HBM."""
    import oracle
    shp = (64, 128, 256)
    st = synth.blob_stack(shp, 50, 0, device="cuda")
    gpu = _b2b_ms(torch, lambda: dsk.deskew(st, 30.0, 0.4, 0.115), 50)
    host = st.cpu().numpy()
    offs = oracle.offsets_uniform(shp[0], oracle.shift_px(30.0, 0.4, 0.115))
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.deskew(host, offs)
        ts.append((time.perf_counter() - t0) * 1e3)
    return {"workload": "64x128x256 uint16, 30 deg, W=446", "gpu_ms": gpu,
            "oracle_ms": statistics.median(ts), "oracle_threads": oracle.threads()}


def copy_ceiling(torch, nbytes=4 << 30, reps=5):
    """Device-to-device copy rate (read + write bytes per second), context only."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del a, b
    return 2 * nbytes / (statistics.median(ts) * 1e-3) / 1e9


def _median_ms(torch, fn, reps):
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


def _one_ms(torch, fn):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1)


def _batch_case(torch, dsk, synth, jobs, seed0, label):
    """One graph launch of a ragged batch against the same stacks as plain
    launches on one stream.  Both write the same output buffers (where
    outputs sit in memory moves this workload's time by up to 20%, so the
    two are compared on one placement) and are timed alternately."""
    from paper_2211_00645_amd.batch import Batch
    stacks, geoms = [], []
    for i, j in enumerate(jobs):
        shp = (j["planes"], j["rows"], j["cols"])
        stacks.append(synth.blob_stack(shp, synth.blobs_for_volume(*shp), seed0 + i,
                                       device="cuda"))
        geoms.append((j["angle_deg"], j["step_um"], j["pixel_um"]))
    torch.cuda.synchronize()
    b = Batch(stacks, geoms)
    tune, mode = b.tune, b.mode
    outs = b.outputs
    alg = sum(2 * o["vol"].numel() // o["width"] * s.shape[2] + 4 * o["vol"].numel()
              + 8 * o["psum"].numel() for o, s in zip(outs, stacks))
    vox = sum(o["vol"].numel() for o in outs)
    b.launch()
    torch.cuda.synchronize()
    # bitwise check, one job at a time against a plain launch
    same = True
    for s, g, o in zip(stacks, geoms, outs):
        r = dsk.deskew(s, *g)
        same = same and all(torch.equal(r[k], o[k]) for k in ("vol", "psum", "pmax"))
        del r
    torch.cuda.empty_cache()

    # each job's frame in the shape the single-stack tuner picks for it (the
    # batch tuner already measured these frames, so this only looks them up)
    job_tunes = [dsk.autotune(s, *g, out=o, reps=3)["tune"] for s, g, o in zip(stacks, geoms, outs)]

    def plain():
        for s, g, o in zip(stacks, geoms, outs):
            dsk.deskew(s, *g, out=o)

    def plain_tuned():
        for s, g, o, t in zip(stacks, geoms, outs, job_tunes):
            dsk.deskew(s, *g, out=o, tune=t)
    plain()
    plain_tuned()
    t_graph, t_plain, t_tuned = [], [], []
    for _ in range(6):
        t_graph.append(_one_ms(torch, b.launch))
        t_plain.append(_one_ms(torch, plain))
        t_tuned.append(_one_ms(torch, plain_tuned))
    ms_graph, ms_plain = statistics.median(t_graph), statistics.median(t_plain)
    ms_tuned = statistics.median(t_tuned)
    b.close()
    del b, outs, stacks
    torch.cuda.empty_cache()
    return {"workload": label,
            "graph_ms": ms_graph, "plain_launches_ms": ms_plain,
            "speedup": ms_plain / ms_graph, "plain_tuned_launches_ms": ms_tuned,
            "speedup_vs_tuned": ms_tuned / ms_graph, "gbs_graph": alg / ms_graph / 1e6,
            "voxels_per_s_graph": vox / ms_graph * 1e3, "algorithmic_bytes": alg,
            "bitwise_equal": same, "mode": mode, "tune": tune,
            "timing": "graph replays, plain launches in the library default shape and "
                      "plain launches in each job's tuned shape alternate, 6 each, on the "
                      "same output buffers; medians"}


def bench_batch(torch, dsk, synth):
    """The 64-stack ragged batch (planes 50-400, rows 256/512/1024, cols
    512-2048), and 256 small ragged stacks (the same draw scaled by 1/8)
    where each plain launch is short and launch overhead counts."""
    big = _batch_case(torch, dsk, synth, synth.ragged_jobs(64, seed=0), 1000,
                      "64 ragged uint16 stacks (planes 50-400, rows 256/512/1024, "
                      "cols 512-2048, 30/35/45 deg), seed 0")
    small = _batch_case(torch, dsk, synth, synth.ragged_jobs(256, seed=1, scale=0.125), 5000,
                        "256 small ragged uint16 stacks (the same draw scaled by 1/8: planes "
                        "7-50, rows 32/64/128, cols 64-256), seed 1")
    big["small_stacks"] = small
    return big


def _b2b_ms(torch, fn, reps):
    """Average time per call of `reps` calls back to back (after 3 warm-up
    calls): kernel time without the host's launch latency."""
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


PROJ_PMC_SUMMARY = os.path.join(ROOT, "profiles", "projections_512x512x2048_pmc.md")


def bench_projections(torch, dsk, stack):
    """The live view alone (Fig. 2d): sum and maximum projections of the
    512 x 512 x 2048 stack without writing the volume, calls back to back,
    in the library default shape and in the shape the tuner picks for this
    frame (as the forward's headline).  One launch reads the stack once and
    writes the two projections."""
    w, b = dsk.plan((N, R, C), shift=dsk.shift_px(ANGLE, STEP, PIXEL))
    out = {"psum": torch.empty((R, w), dtype=torch.float32, device=stack.device),
           "pmax": torch.empty((R, w), dtype=torch.float32, device=stack.device)}
    reps = 50

    def call(tune):
        return lambda: dsk.deskew(stack, ANGLE, STEP, PIXEL, vol=False, out=out, tune=tune)

    ms_default = _b2b_ms(torch, call(None), reps)
    tuned = dsk.autotune(stack, ANGLE, STEP, PIXEL, vol=False, out=out, reps=16)
    ms = _b2b_ms(torch, call(tuned["tune"]), reps)
    alg = 2 * N * R * C + 8 * R * w
    achieved = alg / (ms * 1e-3) / 1e9
    return {"workload": "sum + max projections only (no volume), 512x512x2048 uint16 stack, "
                        "35 deg, launch shape tuned for the frame",
            "ms": ms, "ms_default_shape": ms_default, "launch_shape": tuned["tune"],
            "algorithmic_bytes": alg, "input_voxels_per_s": N * R * C / ms * 1e3,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic(PROJ_PMC_SUMMARY)},
            "timing": f"{reps} launches back to back between two events on the launch stream"}


def bench_autograd(torch, dsk, synth):
    """Forward (float32, tuned shape) + fused backward on 256 x 512 x 1024,
    frame 1793; calls back to back."""
    n, r, c, w = 256, 512, 1024, 1793
    st = synth.blob_stack((n, r, c), 2000, 4, device="cuda", dtype="f32")
    offs = torch.arange(n, dtype=torch.float64, device="cuda") * dsk.shift_px(30.0, STEP, PIXEL)
    out = {"vol": torch.empty((n, r, w), device="cuda")}
    gd = torch.empty((n, r, w), device="cuda").uniform_()
    fwd = _b2b_ms(torch, lambda: dsk.deskew(st, offsets=offs, origin=0, width=w, out=out,
                                             psum=False, pmax=False, tune="auto"), 20)
    bwd = _b2b_ms(torch, lambda: dsk.backward(st, gd, offs, 0), 20)
    del out, gd
    # calibration: recover 32 deg from 30 deg, the target being the
    # library's own deskew at 32 deg on the same frame
    from paper_2211_00645_amd import autograd as ag
    a32 = torch.tensor(32.0, dtype=torch.float64, device="cuda")
    tgt = dsk.deskew(st, offsets=ag.offsets_from_angle(a32, n, STEP, PIXEL), origin=0,
                     width=w, psum=False, pmax=False)["vol"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    angle, hist = ag.calibrate_angle(st, tgt, 30.0, STEP, PIXEL, 0, w)
    torch.cuda.synchronize()
    cal_s = time.perf_counter() - t0
    del st, tgt
    torch.cuda.empty_cache()
    fb = 4 * n * r * c + 4 * n * r * w
    # backward: the gradient volume's band that the stack maps to (n r c of
    # its n r w values) and the stack read once, the adjoint written once
    bb = 12 * n * r * c
    return {"workload": "float32 256x512x1024, frame 1793",
            "forward_ms": fwd, "forward_gbs": fb / fwd / 1e6,
            "backward_ms": bwd, "backward_gbs": bb / bwd / 1e6,
            "calibration": {"from_deg": 30.0, "target_deg": 32.0, "final_deg": angle,
                            "steps": len(hist), "seconds": cal_s}}


def bench_view(torch, dsk, synth):
    """Shear-warp views of the 512 x 512 x 2048 stack: projections of the
    re-sheared stack (no volume) plus the column stretch, per view angle."""
    st = synth.blob_stack((N, R, C), BLOBS, SEED, device="cuda")
    res = {"workload": "shear-warp views of the 512x512x2048 uint16 stack, 35 deg"}
    for theta in (0.0, 20.0, ANGLE):
        g = dsk.view_plan((N, R, C), theta, ANGLE, STEP, PIXEL)
        ws = torch.empty((R * g["proj_width"] * 2,), dtype=torch.float32, device="cuda")
        ms = _median_ms(torch, lambda: dsk.view(st, theta, ANGLE, STEP, PIXEL, workspace=ws), 10)
        alg = 2 * N * R * C + 16 * R * g["proj_width"] + 8 * R * g["width"]
        res[f"theta_{theta:g}"] = {"ms": ms, "gbs": alg / ms / 1e6, "shear_px": g["shear"],
                                   "stretch": g["stretch"], "proj_width": g["proj_width"],
                                   "view_width": g["width"], "algorithmic_bytes": alg}
    del st
    torch.cuda.empty_cache()
    return res


def bench_affine(torch, dsk, synth):
    """Real-space (affine) deskew of the 512 x 512 x 2048 stack onto a
    0.115 um scan grid (3455 x 512 x 2048 float32 output)."""
    st = synth.blob_stack((N, R, C), BLOBS, SEED, device="cuda")
    y0, ny = dsk.affine_plan((N, R, C), ANGLE, STEP, PIXEL, PIXEL)
    out = torch.empty((ny, R, C), dtype=torch.float32, device="cuda")
    ms = _median_ms(torch, lambda: dsk.affine(st, ANGLE, STEP, PIXEL, PIXEL, out=out), 5)
    alg = 2 * N * R * C + 4 * ny * R * C
    del st, out
    torch.cuda.empty_cache()
    return {"workload": "affine deskew of the 512x512x2048 uint16 stack, 35 deg, dy 0.115 um",
            "ny": ny, "ms": ms, "gbs": alg / ms / 1e6, "algorithmic_bytes": alg,
            "voxels_per_s": ny * R * C / ms * 1e3}


def bench_rolling(torch, dsk, synth):
    """Rolling display mode: time per image update (remap of one image,
    max-tree path, running sum, projections), at the paper's live region
    (50 images of 1304 x 87 px spread over 3652 px) and at the benchmark
    stack's shape (512 images of 512 x 2048)."""
    from paper_2211_00645_amd.rolling import RollingView
    res = {"workload": "rolling update, one image per call"}
    for name, (n, r, c), kw in (("paper_1304x87x50", (50, 1304, 87),
                                 {"shift_px": (3652 - 87) / 49}),
                                ("stack_512x512x2048", (N, R, C),
                                 {"angle_deg": ANGLE, "step_um": STEP, "pixel_um": PIXEL})):
        st = synth.blob_stack((n, r, c), 50, 21, device="cuda")
        rv = RollingView(n, r, c, **kw)
        for i in range(n):
            rv.update(i, st[i])
        torch.cuda.synchronize()
        k = [0]

        def one():
            rv.update(k[0] % n, st[k[0] % n])
            k[0] += 1
        ms = _median_ms(torch, one, 50)          # one call, host launch included
        kms = _b2b_ms(torch, one, 100)           # calls back to back
        # bytes per update: the image, the leaf read and written, the FP64
        # running sum read and written, both projections written, and per
        # tree level a sibling read and the parent written
        levels = max(1, math.ceil(math.log2(n))) if n > 1 else 0
        w = rv.width
        alg = 2 * r * c + (8 + 16 + 8 + 8 * levels) * r * w
        res[name] = {"ms_per_image": ms, "images_per_s": 1e3 / ms, "width": w,
                     "kernel_ms": kms, "algorithmic_bytes": alg, "gbs": alg / kms / 1e6}
        del rv, st
        torch.cuda.empty_cache()
    return res


def bench_size_sweep(torch, dsk, synth):
    """Forward time against the number of images N (512 x 2048 images at
    35 deg) and against the output width W (512 images, scan step varied):
    the paper's processing time grows linearly in both (Supp. Table 1).
    Each frame is timed with the library default and with the shape the
    tuner picks for it."""
    res = {"workload": "forward, 512x2048 uint16 images", "vs_planes": [], "vs_width": []}
    st = synth.blob_stack((N, R, C), BLOBS, SEED, device="cuda")

    def one(sub, step):
        w, _ = dsk.plan(tuple(sub.shape), shift=dsk.shift_px(ANGLE, step, PIXEL))
        tuned = dsk.autotune(sub, ANGLE, step, PIXEL, reps=6)["tune"]
        ms_def = _median_ms(torch, lambda: dsk.deskew(sub, ANGLE, step, PIXEL), 10)
        ms = _median_ms(torch, lambda: dsk.deskew(sub, ANGLE, step, PIXEL, tune=tuned), 10)
        alg = algorithmic_bytes(sub.shape[0], R, C, w)
        return {"width": w, "ms_default": ms_def, "ms_tuned": ms,
                "gbs_tuned": alg / ms / 1e6, "tune": tuned}

    for n in (64, 128, 256, 512):
        res["vs_planes"].append(dict(planes=n, **one(st[:n], STEP)))
    for step in (0.1, 0.2, 0.4, 0.8):
        res["vs_width"].append(dict(step_um=step, **one(st, step)))
    del st
    torch.cuda.empty_cache()
    return res


def bench_serving(torch, dsk, synth, n_req, rate, sweep=(), sweep_s=6.0, n_live=400):
    """Poisson arrivals of 2-channel stacks (100-400 x 512/1024 x 1024/2048),
    200 GB budget; continuous batching vs one stack at a time.  The live run
    has ``n_live`` requests (its p99 is then the 4th-worst latency of 400,
    not the 2nd of 200); the burst has ``n_req``."""
    from paper_2211_00645_amd import serving as sv
    pool = {}
    for k, (r, c) in enumerate([(512, 1024), (512, 2048), (1024, 1024), (1024, 2048)]):
        for ch in range(2):
            pool[(r, c, ch)] = synth.blob_stack((400, r, c), synth.blobs_for_volume(400, r, c),
                                                500 + 2 * k + ch, device="cuda")
    torch.cuda.synchronize()
    budget = 200 << 30
    res = {"workload": f"2-channel stacks: {n_live} at Poisson {rate} Hz (live) and {n_req} "
                       f"at once (burst), 200 GiB budget"}
    # one executor: its output arena is reserved once and reused by every run
    ex = sv.GPUExecutor(pool, n_slots=4, arena_bytes=budget)
    # the consumer of a live stream: takes each stack's projections as it
    # completes and lets them go (their pinned buffer returns to the cache)
    def consume(r):
        r.result = None
    # warm-up burst (untimed): fills the pinned-memory cache
    sv.Scheduler(ex, budget, n_slots=4, max_batch=8, on_complete=consume).run(
        sv.make_requests(synth.serving_trace(48, 1e9, 9)))
    for mode in ("live", "burst"):
        r_ = rate if mode == "live" else 1e9
        tr = synth.serving_trace(n_live if mode == "live" else n_req, r_, 7)
        sch = sv.Scheduler(ex, budget, n_slots=4, max_batch=8, on_complete=consume)
        res[mode] = dict(sv.summarize(sch.run(sv.make_requests(tr))), launches=sch.launches,
                         peak_gb=sch.peak_used / 1e9, space_waits=sch.space_waits)
        res[mode + "_plain"] = sv.summarize(sv.run_plain(ex, sv.make_requests(tr),
                                                         on_complete=consume))
        log(f"serving {mode}: p50 {res[mode]['latency_p50_ms']:.2f} ms p99 "
            f"{res[mode]['latency_p99_ms']:.2f} ms; plain p99 "
            f"{res[mode + '_plain']['latency_p99_ms']:.2f} ms")
    if sweep:
        # each arrival rate: the same trace served and one stack at a time
        res["sweep"] = {}
        for lam in sweep:
            n = int(max(30, round(lam * sweep_s)))
            tr = synth.serving_trace(n, lam, 11)
            sch = sv.Scheduler(ex, budget, n_slots=4, max_batch=8, on_complete=consume)
            served = dict(sv.summarize(sch.run(sv.make_requests(tr))), launches=sch.launches)
            plain = sv.summarize(sv.run_plain(ex, sv.make_requests(tr), on_complete=consume))
            res["sweep"][f"{lam:g}Hz"] = {"requests": n, "served": served, "plain": plain}
            log(f"serving {lam:g} Hz x {n}: p99 {served['latency_p99_ms']:.2f} ms "
                f"(max {served['latency_max_ms']:.2f}); plain p99 {plain['latency_p99_ms']:.2f} "
                f"(max {plain['latency_max_ms']:.2f})")
    del pool, ex
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # 10 untimed steps: the first launches after the device has idled run
    # slower for about ten launches while its clocks ramp, which throws a
    # paced launch off its schedule
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--extras",
                    default="projections,batch,autograd,view,affine,rolling,sizes,serving",
                    help="comma list of extra measurements (projections, batch, autograd, view, "
                         "affine, rolling, sizes, serving) or none")
    ap.add_argument("--tune", default="auto",
                    help="launch shape of the timed forward: auto (the library's tuner, run "
                         "once before the warm-up) or default (the library default)")
    ap.add_argument("--serve-requests", type=int, default=200, help="burst size")
    ap.add_argument("--serve-live-requests", type=int, default=400,
                    help="requests of the live (Poisson) run")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-sweep", default="5,10,20,50",
                    help="comma list of arrival rates (Hz) also run live, served and one "
                         "stack at a time, for about --serve-seconds each ('' to skip)")
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process on one GPU.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2211_00645_amd as dsk
    from paper_2211_00645_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"device {torch.cuda.get_device_name(dev)}; generating {N}x{R}x{C} u16 stack")
    stack = synth.blob_stack((N, R, C), BLOBS, SEED, device=dev)
    torch.cuda.synchronize()

    w, b = dsk.plan((N, R, C), shift=dsk.shift_px(ANGLE, STEP, PIXEL))
    outs = {"vol": torch.empty((N, R, w), dtype=torch.float32, device=dev),
            "psum": torch.empty((R, w), dtype=torch.float32, device=dev),
            "pmax": torch.empty((R, w), dtype=torch.float32, device=dev)}

    if args.tune == "auto":
        log("tuning the launch shape for this frame")
        tuned = dsk.autotune(stack, ANGLE, STEP, PIXEL, out=outs, reps=16)
        shape = tuned["tune"]
        log(f"launch shape {shape} ({tuned['ms']:.4f} ms mean while tuning)")
    elif args.tune == "default":
        shape = None
    else:
        print(f"--tune must be auto or default (got {args.tune})", file=sys.stderr)
        sys.exit(2)

    def step():
        return dsk.deskew(stack, ANGLE, STEP, PIXEL, out=outs, tune=shape)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms_per_step = wall * 1e3 / args.steps
    avg_kern_ms = sum(kern_ms) / len(kern_ms)

    vox = N * R * w
    alg = algorithmic_bytes(N, R, C, w)
    achieved = alg / (avg_kern_ms * 1e-3) / 1e9
    log(f"kernel avg {avg_kern_ms:.4f} ms (median {statistics.median(kern_ms):.4f}); "
        f"{achieved:.0f} GB/s; wall {ms_per_step:.4f} ms/step")

    extras = [e for e in args.extras.split(",") if e and e != "none"]
    ext = {}
    if "projections" in extras:
        log("projections only (live view)")
        ext["projections"] = bench_projections(torch, dsk, stack)
        pr = ext["projections"]
        log(f"projections: {pr['ms']:.4f} ms, {pr['roofline']['achieved']:.0f} GB/s "
            f"({pr['roofline']['frac']:.3f} of peak) in {pr['launch_shape']}; "
            f"default shape {pr['ms_default_shape']:.4f} ms")

    copy_gbs = copy_ceiling(torch)
    log(f"device copy ceiling {copy_gbs:.0f} GB/s")

    cpu = None
    del outs
    torch.cuda.synchronize()
    config1 = None
    if args.cpu_seconds > 0:
        host = stack.cpu().numpy()
        cpu = cpu_baseline(host, args.cpu_seconds)
        cpu.pop("seconds", None)
        del host
        config1 = config1_times(torch, dsk, synth)
    del stack
    torch.cuda.empty_cache()

    if "batch" in extras:
        log("batch: 64 ragged stacks")
        ext["batch"] = bench_batch(torch, dsk, synth)
        bb, bs = ext["batch"], ext["batch"]["small_stacks"]
        log(f"batch: graph {bb['graph_ms']:.2f} ms ({bb['mode']}) vs plain "
            f"{bb['plain_launches_ms']:.2f} ms, plain tuned {bb['plain_tuned_launches_ms']:.2f} "
            f"ms; small stacks: graph {bs['graph_ms']:.3f} ms ({bs['mode']}) vs plain "
            f"{bs['plain_launches_ms']:.3f} ms, plain tuned {bs['plain_tuned_launches_ms']:.3f} ms")
    if "autograd" in extras:
        log("autograd: forward + backward")
        ext["autograd"] = bench_autograd(torch, dsk, synth)
    if "view" in extras:
        log("view: shear-warp rotated views")
        ext["view"] = bench_view(torch, dsk, synth)
    if "affine" in extras:
        log("affine: real-space deskew")
        ext["affine"] = bench_affine(torch, dsk, synth)
        log(f"affine: {ext['affine']['ms']:.3f} ms, {ext['affine']['gbs']:.0f} GB/s")
    if "rolling" in extras:
        log("rolling: per-image update")
        ext["rolling"] = bench_rolling(torch, dsk, synth)
    if "sizes" in extras:
        log("size sweep: time vs images and width")
        ext["size_sweep"] = bench_size_sweep(torch, dsk, synth)
    if "serving" in extras:
        log("serving")
        ext["serving"] = bench_serving(torch, dsk, synth, args.serve_requests, args.serve_rate,
                                       [float(v) for v in args.serve_sweep.split(",") if v],
                                       args.serve_seconds, args.serve_live_requests)

    rec = {
        "metric": METRIC,
        "value": vox / (ms_per_step * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (Poisson(100) background + 2000 Gaussian spots, seed 2)",
        "config": {"workload": "deskew+sum/max projection, 512x512x2048 uint16 stack, 35 deg, "
                               "0.4 um step, 0.115 um pixel",
                   "planes": N, "rows": R, "cols": C, "out_width": w, "origin": b,
                   "input": "u16", "volume": "f32", "sum_accumulation": "f64",
                   "launch_shape": shape or "library default",
                   "parallelism": "single GPU"},
        "input_voxels_per_s": N * R * C / (ms_per_step * 1e-3),
        "hbm_gbs": alg / (ms_per_step * 1e-3) / 1e9,
        "kernel_ms_avg": avg_kern_ms,
        "kernel_ms_median": statistics.median(kern_ms),
        "algorithmic_bytes": alg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic()},
        "copy_ceiling_gbs": copy_gbs,
        "cpu_baseline": cpu,
    }
    if config1 is not None:
        rec["config1"] = config1
    if "serving" in ext:
        rec["latency_p99_ms_live"] = ext["serving"]["live"]["latency_p99_ms"]
    # the extras never replace a field of the line's contract
    assert not set(ext) & set(rec), sorted(set(ext) & set(rec))
    rec.update(ext)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
