"""Ragged batches: many uint16 stacks of different shapes and geometries
deskewed by ONE graph launch.

The graph holds either one persistent kernel over all jobs or one plain
paced launch per job (default shape, or each job frame's tuned shape).  The
library's autotuner times the persistent kernel's candidate shapes (threads
per workgroup, columns per thread, plane unroll, pacing) and the per-job
modes on the batch's own buffers, keeps the fastest, and caches the choice
per device architecture and batch shape class in a JSON file
(``DSK_TUNE_CACHE``).  Each job's outputs are bitwise
identical to its own single-stack call in either mode.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import torch

from . import _lib as L
from . import api


def _job(stack, shift, origin, width, vol, psum, pmax, offsets_dev=None):
    n, r, c = (int(v) for v in stack.shape)
    j = L.Job()
    j.in_ = stack.data_ptr()
    j.dims = L.Dims(n, r, c)
    j.offsets_dev = None if offsets_dev is None else offsets_dev.data_ptr()
    j.shift_px = float(shift)
    j.origin = int(origin)
    j.out_width = int(width)
    j.vol = None if vol is None else vol.data_ptr()
    j.psum = None if psum is None else psum.data_ptr()
    j.pmax = None if pmax is None else pmax.data_ptr()
    return j


def plan_job(stack, angle_deg, step_um, pixel_um, vol=True, psum=True, pmax=True, out=None):
    """Allocate (or take from ``out``) the outputs of one stack and return
    (job record, outputs dict).  Geometry as in ``api.deskew``."""
    api._check_stack(stack, (torch.uint16,))
    n, r, c = (int(v) for v in stack.shape)
    shift = api.shift_px(angle_deg, step_um, pixel_um)
    w, b = api.plan((n, r, c), shift=shift)
    out = dict(out or {})
    res = {"origin": b, "width": w}
    for key, want, shp in (("vol", vol, (n, r, w)), ("psum", psum, (r, w)),
                           ("pmax", pmax, (r, w))):
        if want:
            t = out.get(key)
            if t is None:
                t = torch.empty(shp, dtype=torch.float32, device=stack.device)
            res[key] = t
    job = _job(stack, shift, b, w, res.get("vol"), res.get("psum"), res.get("pmax"))
    return job, res


@contextlib.contextmanager
def _tune_cache(path):
    """Point the library's tune cache (the DSK_TUNE_CACHE variable, read at
    each lookup) at ``path`` for one call, then restore the previous value:
    a batch's cache file does not leak into later calls of the process."""
    if path is None:
        yield
        return
    key = "DSK_TUNE_CACHE"
    prev = os.environ.get(key)
    os.environ[key] = str(path)
    try:
        yield
    finally:
        if prev is None:
            os.environ.pop(key, None)
        else:
            os.environ[key] = prev


class Batch:
    """One graph launch over ragged stacks (persistent kernel or one launch
    per job, see :attr:`mode`).

    ``stacks``: list of contiguous uint16 CUDA tensors [planes][rows][cols];
    ``geoms``: list of (angle_deg, step_um, pixel_um).  ``tune``: launch
    shape dict, or None to autotune (which runs the batch a few times).
    Outputs are in ``self.outputs[i]`` (``vol``, ``psum``, ``pmax``,
    ``origin``, ``width``).
    """

    def __init__(self, stacks, geoms, vol=True, psum=True, pmax=True, tune=None,
                 cache_path=None, stream=None):
        if len(stacks) != len(geoms) or not stacks:
            raise ValueError("need one geometry per stack")
        self.stacks = list(stacks)
        self.outputs = []
        jobs = (L.Job * len(stacks))()
        for i, (s, g) in enumerate(zip(stacks, geoms)):
            jobs[i], res = plan_job(s, *g, vol=vol, psum=psum, pmax=pmax)
            self.outputs.append(res)
        self._jobs = jobs
        handle = ctypes.c_void_p()
        tn = api._tune(tune)
        with _tune_cache(cache_path):
            st = L.lib().dsk_batch_create(jobs, len(stacks), ctypes.byref(tn) if tn else None,
                                          api._stream(stream), ctypes.byref(handle))
        L.check(st, "dsk_batch_create")
        self._h = handle

    @property
    def tune(self):
        t = L.Tune()
        ms = ctypes.c_double()
        L.check(L.lib().dsk_batch_get_tune(self._h, ctypes.byref(t), ctypes.byref(ms)),
                "dsk_batch_get_tune")
        return dict(t.as_dict(), tuned_ms=ms.value)

    @property
    def mode(self):
        """"persistent" (one kernel over all jobs), "per_job" (one plain
        launch per job, default shape) or "per_job_tuned" (one plain launch
        per job in its frame's tuned shape), as the autotuner chose
        (persistent when a shape was given)."""
        m = ctypes.c_int()
        L.check(L.lib().dsk_batch_get_mode(self._h, ctypes.byref(m)), "dsk_batch_get_mode")
        return {0: "persistent", 1: "per_job", 2: "per_job_tuned"}[m.value]

    def launch(self, stream=None, graph=True):
        """Enqueue the whole batch (graph replay, or a direct launch)."""
        if self._h is None:
            raise RuntimeError("batch destroyed")
        fn = L.lib().dsk_batch_launch if graph else L.lib().dsk_batch_launch_direct
        L.check(fn(self._h, api._stream(stream)), "dsk_batch_launch")

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lib().dsk_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class JobLauncher:
    """Launch per-call job lists with one persistent kernel (the serving
    path): the job table is encoded into pinned host memory and copied to
    the device on the launch stream, so nothing is allocated per launch.
    ``max_jobs`` bounds the table size; ``slots`` tables rotate so a table
    is not overwritten while an earlier copy may still be pending."""

    def __init__(self, max_jobs=64, slots=4, device="cuda"):
        nb = int(L.lib().dsk_jobs_table_bytes(int(max_jobs)))
        self.max_jobs = int(max_jobs)
        self.nbytes = nb
        self.host = [torch.empty(nb, dtype=torch.uint8, pin_memory=True) for _ in range(slots)]
        self.dev = [torch.empty(nb, dtype=torch.uint8, device=device) for _ in range(slots)]
        self.events = [None] * slots
        self.k = 0

    def launch(self, jobs, tune=None, stream=None):
        n = len(jobs)
        if n == 0:
            return
        if n > self.max_jobs:
            raise ValueError(f"{n} jobs > max_jobs {self.max_jobs}")
        i = self.k % len(self.host)
        self.k += 1
        if self.events[i] is not None:
            self.events[i].synchronize()      # that table's copy has finished
        arr = (L.Job * n)(*jobs)
        tn = api._tune(tune)
        s = stream if stream is not None else torch.cuda.current_stream()
        st = L.lib().dsk_jobs_launch(arr, n, ctypes.c_void_p(self.host[i].data_ptr()),
                                     ctypes.c_void_p(self.dev[i].data_ptr()), self.nbytes,
                                     ctypes.byref(tn) if tn else None, api._stream(s))
        L.check(st, "dsk_jobs_launch")
        ev = torch.cuda.Event()
        ev.record(s)
        self.events[i] = ev
