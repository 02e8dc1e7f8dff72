"""The allocation-free backward (dsk_backward_f32_noalloc) against the
backward that takes a caller workspace (dsk_backward_f32), through the C
ABI: two calls in a row on one device, the second on a smaller stack, so
the second reuses the library's device array after a larger call.  Both
entry points run the same kernels, so the results must be bitwise equal;
the small case is also held to the oracle at the adjoint's 1e-5 bar."""
import numpy as np
import pytest
import torch

import oracle
from paper_2211_00645_amd import _lib as L
from paper_2211_00645_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _vp(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _both(stack, gd, offs, origin):
    """(grad_in, grad_offsets) from the workspace entry point and from the
    allocation-free one, on the same inputs."""
    n, r, c = stack.shape
    w = gd.shape[2]
    dims = L.Dims(n, r, c)
    lib = L.lib()
    wsb = int(lib.dsk_shear_grad_workspace_bytes(dims))
    ws = torch.empty((max(1, wsb // 8),), dtype=torch.float64, device=DEV)
    out = []
    for noalloc in (False, True):
        gi = torch.full((n, r, c), float("nan"), dtype=torch.float32, device=DEV)
        go = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
        if noalloc:
            st = lib.dsk_backward_f32_noalloc(_vp(stack), _vp(gd), dims, _vp(offs), int(origin),
                                              int(w), _vp(gi), _vp(go), _stream())
        else:
            st = lib.dsk_backward_f32(_vp(stack), _vp(gd), dims, _vp(offs), int(origin), int(w),
                                      _vp(gi), _vp(go), _vp(ws), wsb, _stream())
        assert st == L.DSK_OK, L.status_string(st)
        torch.cuda.synchronize()
        out.append((gi.cpu(), go.cpu()))
    return out


def test_noalloc_backward_matches_workspace_backward_twice():
    # call 1: the 256 x 512 x 1024 float32 stack, frame 1793 at 30 degrees
    print("noalloc call 1: 256x512x1024, width 1793", flush=True)
    n, r, c, w = 256, 512, 1024, 1793
    stack = synth.blob_stack((n, r, c), 2000, 4, device=DEV, dtype="f32")
    offs = (torch.arange(n, dtype=torch.float64) * oracle.shift_px(30.0, 0.4, 0.115)).to(DEV)
    gen = torch.Generator(device=DEV).manual_seed(11)
    gd = torch.rand((n, r, w), generator=gen, device=DEV) * 2 - 1
    (gi_ws, go_ws), (gi_na, go_na) = _both(stack, gd, offs, 0)
    assert torch.equal(gi_ws, gi_na)
    assert torch.equal(go_ws, go_na)
    assert torch.isfinite(go_na).all()
    del stack, gd
    torch.cuda.empty_cache()

    # call 2: a smaller ragged stack with jittered offsets, after the large one
    print("noalloc call 2: 23x17x301, jittered offsets", flush=True)
    rng = np.random.default_rng(7)
    n, r, c = 23, 17, 301
    s = synth.blob_stack((n, r, c), 40, 5, dtype="f32").numpy()
    off = np.cumsum(np.r_[0.0, rng.uniform(0.2, 5.0, n - 1)])
    b, w = oracle.frame(off, c)
    gdh = rng.uniform(-1, 1, (n, r, w)).astype(np.float32)
    (gi_ws, go_ws), (gi_na, go_na) = _both(torch.from_numpy(s).to(DEV),
                                           torch.from_numpy(gdh).to(DEV),
                                           torch.from_numpy(off).to(DEV), b)
    assert torch.equal(gi_ws, gi_na)
    assert torch.equal(go_ws, go_na)
    ref_gi = oracle.adjoint(gdh, off, b, c).astype(np.float64)
    mag = oracle.adjoint(np.abs(gdh), off, b, c, as_f64=True)
    assert (np.abs(gi_na.numpy().astype(np.float64) - ref_gi) <= 1e-5 * mag + 1e-30).all()
    ref_go = oracle.shear_grad(s, gdh, off, b)
    bound = 2.0 * np.abs(s).max() * np.abs(gdh).astype(np.float64).sum(axis=(1, 2))
    assert (np.abs(go_na.numpy() - ref_go) <= 1e-5 * bound).all()


def test_noalloc_adjoint_only_needs_no_array():
    print("noalloc adjoint only: 9x5x64", flush=True)
    n, r, c = 9, 5, 64
    rng = np.random.default_rng(3)
    off = np.arange(n, dtype=np.float64) * 2.5
    b, w = oracle.frame(off, c)
    gdh = rng.uniform(-1, 1, (n, r, w)).astype(np.float32)
    gd = torch.from_numpy(gdh).to(DEV)
    offs = torch.from_numpy(off).to(DEV)
    gi = torch.empty((n, r, c), dtype=torch.float32, device=DEV)
    st = L.lib().dsk_backward_f32_noalloc(None, _vp(gd), L.Dims(n, r, c), _vp(offs), int(b),
                                          int(w), _vp(gi), None, _stream())
    assert st == L.DSK_OK, L.status_string(st)
    torch.cuda.synchronize()
    ref = oracle.adjoint(gdh, off, b, c).astype(np.float64)
    mag = oracle.adjoint(np.abs(gdh), off, b, c, as_f64=True)
    assert (np.abs(gi.cpu().numpy().astype(np.float64) - ref) <= 1e-5 * mag + 1e-30).all()
