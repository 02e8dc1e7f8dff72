"""The checking build (libdeskew_bounds.so, compiled with DSK_CHECK_BOUNDS=1)
sends every global address of the forward (with and without the volume,
every launch-shape family: scalar and vector kernels, one or two groups per
lane, 64/128/256-thread workgroups, 1/2/4-plane pipelines, paced), the
persistent batch kernel and the backward through a check against its
buffer's extent.  Run over ragged, stack-end and strided-channel shapes,
no address lies outside its buffer.  The checking library runs in a child
process (one library per process)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_00645_amd", "libdeskew_bounds.so")

CHILD = r"""
import ctypes, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_2211_00645_amd as dsk
from paper_2211_00645_amd import _lib as L, synth
from paper_2211_00645_amd.batch import Batch

lib = L.lib()
cnt = ctypes.c_ulonglong(0)
assert lib.dsk_debug_bounds_violations(ctypes.byref(cnt), 1) == 1, "not a checking build"
DEV = "cuda:0"

def say(m):
    print(m, flush=True)

def offsets(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "frac":
        return np.arange(n) * 2.718281828
    if kind == "neg":
        return np.arange(n) * -1.4142135
    if kind == "jitter":
        return np.cumsum(np.r_[0.0, rng.uniform(0.5, 3.5, n - 1)])
    if kind == "shuffle":
        return rng.permutation(n).astype(np.float64) * 5.3 + rng.uniform(0, 1, n)
    return np.zeros(n)

SHAPES = [(1, 3, 17, "frac"), (7, 5, 33, "neg"), (13, 9, 257, "frac"), (33, 7, 513, "jitter"),
          (4, 4, 7, "frac"), (9, 12, 300, "neg"), (2, 2, 2, "frac"), (150, 6, 400, "shuffle"),
          (200, 8, 300, "frac"), (1, 4, 64, "frac"), (65, 4, 64, "frac"), (129, 4, 96, "neg"),
          (70, 16, 256, "zero"), (64, 40, 512, "frac")]
TUNES = [None] + [dict(block=b, per_thread=j, nt_store=1, unroll=u, pace_gbs=p)
                  for b, j, u, p in ((64, 1, 1, 0), (128, 2, 1, 0), (64, 4, 1, 0), (64, 4, 2, 5800),
                                     (256, 4, 4, 0), (64, 8, 2, 0), (128, 8, 4, 9000))]
for n, r, c, kind in SHAPES:
    for dt in ("u16", "f32"):
        st = synth.blob_stack((n, r, c), max(1, n * r * c // 20000), 3, device=DEV,
                              **({} if dt == "u16" else {"dtype": "f32"}))
        off = offsets(kind, n, 5)
        for t in TUNES:
            dsk.deskew(st, offsets=off, tune=t)
            dsk.deskew(st, offsets=off, tune=t, vol=False)
        dsk.deskew(st, offsets=off, psum=False, pmax=False)
    say(f"forward {n}x{r}x{c} {kind}")

frames = synth.blob_stack((30, 16, 401), 40, 11, device=DEV)
dsk.deskew_channels(frames, (1, 203), 197, 35.0, 0.4, 0.115)
frames = synth.blob_stack((48, 64, 512), 40, 12, device=DEV)
dsk.deskew_channels(frames, (0, 256), 256, 35.0, 0.4, 0.115)
dsk.deskew_channels(frames, (0, 256), 256, 35.0, 0.4, 0.115, vol=False)
say("channels")

jobs = synth.ragged_jobs(10, seed=3, scale=0.12)
stacks = [synth.blob_stack((j["planes"], j["rows"], j["cols"]), 30, 20 + i, device=DEV)
          for i, j in enumerate(jobs)]
geoms = [(j["angle_deg"], j["step_um"], j["pixel_um"]) for j in jobs]
for t in (dict(block=64, per_thread=4, unroll=2, nt_store=1),
          dict(block=256, per_thread=8, unroll=4, nt_store=1, pace_gbs=5500),
          dict(block=128, per_thread=1, unroll=1, nt_store=0)):
    for vol in (True, False):
        b = Batch(stacks, geoms, vol=vol, tune=t)
        b.launch()
        torch.cuda.synchronize()
        b.close()
say("batch")

for n, r, c in ((23, 17, 301), (40, 8, 256), (5, 3, 64)):
    st = synth.blob_stack((n, r, c), 20, 7, device=DEV, dtype="f32")
    offs = torch.from_numpy(np.arange(n) * 1.7 + 0.3).to(DEV)
    w = dsk.plan((n, r, c), offsets=offs.cpu().numpy())[0]
    gd = torch.rand((n, r, w), device=DEV)
    dsk.backward(st, gd, offs, 0)
    dsk.backward(st, gd, offs, 0, grad_offsets=False)
    dsk.backward(st, gd, offs, 0, grad_in=False)
say("backward")

torch.cuda.synchronize()
assert lib.dsk_debug_bounds_violations(ctypes.byref(cnt), 0) == 1
print(f"violations {cnt.value}", flush=True)
"""


def test_no_address_outside_its_buffer():
    assert os.path.exists(LIB), ("the checking library is missing: "
                                 "python -m paper_2211_00645_amd.build --bounds")
    env = dict(os.environ, DSK_LIB=LIB)
    r = subprocess.run([sys.executable, "-u", "-c", CHILD, ROOT], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    print(r.stdout[-4000:])
    print(r.stderr[-4000:])
    assert r.returncode == 0, "child failed"
    assert "violations 0" in r.stdout
