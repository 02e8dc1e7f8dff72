"""Torch-facing API over libdeskew.so.

PyTorch provides device memory and the current stream; the deskew itself runs
in the library's kernels.  Stacks are [planes][rows][cols] CUDA tensors
(uint16 or float32, contiguous); outputs are float32 CUDA tensors:
``vol`` [planes][rows][width], ``psum`` and ``pmax`` [rows][width].
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dims(shape):
    n, r, c = (int(v) for v in shape)
    return L.Dims(n, r, c)


def _check_stack(x, dtypes=(torch.uint16, torch.float32)):
    if not isinstance(x, torch.Tensor) or x.dim() != 3:
        raise ValueError("stack must be a 3-D tensor [planes][rows][cols]")
    if not x.is_cuda:
        raise ValueError("stack must be a CUDA (HIP) tensor")
    if x.dtype not in dtypes:
        raise TypeError(f"stack dtype {x.dtype} not in {dtypes}")
    if not x.is_contiguous():
        raise ValueError("stack must be contiguous")


def _tune(t):
    if t is None:
        return None
    if isinstance(t, L.Tune):
        return t
    return L.Tune(int(t.get("block", 64)), int(t.get("per_thread", 4)),
                  int(t.get("nt_store", 1)), int(t.get("unroll", 2)),
                  int(t.get("wg_per_cu", 0)), int(t.get("pace_gbs", 0)))


def shift_px(angle_deg: float, step_um: float, pixel_um: float) -> float:
    """Per-image shift in pixels (Eq. 1), computed by the library in FP64."""
    out = ctypes.c_double()
    L.check(L.lib().dsk_shift_px(L.Geom(angle_deg, step_um, pixel_um), ctypes.byref(out)),
            "dsk_shift_px")
    return out.value


def plan(shape, shift=None, offsets=None):
    """(width W, origin b) of the remap's larger image for a stack shape."""
    w, b = ctypes.c_int64(), ctypes.c_int64()
    if offsets is not None:
        o = np.ascontiguousarray(
            offsets.detach().cpu().numpy() if isinstance(offsets, torch.Tensor) else offsets,
            np.float64)
        if o.shape != (int(shape[0]),):
            raise ValueError("offsets must have one entry per plane")
        ptr = o.ctypes.data_as(ctypes.c_void_p)
        st = L.lib().dsk_plan(_dims(shape), ptr, 0.0, ctypes.byref(w), ctypes.byref(b))
    else:
        st = L.lib().dsk_plan(_dims(shape), None, float(shift), ctypes.byref(w), ctypes.byref(b))
    L.check(st, "dsk_plan")
    return int(w.value), int(b.value)


def _offsets_dev(offsets, device):
    if isinstance(offsets, torch.Tensor):
        o = offsets.detach().to(device=device, dtype=torch.float64).contiguous()
    else:
        o = torch.as_tensor(np.asarray(offsets, np.float64), device=device)
    return o


def _setup(stack, angle_deg, step_um, pixel_um, offsets, origin, width, vol, psum, pmax, out):
    """Geometry, frame and output tensors shared by deskew() and autotune()."""
    _check_stack(stack)
    dev = stack.device
    shape = tuple(stack.shape)
    shift = None
    if offsets is None:
        if None in (angle_deg, step_um, pixel_um):
            raise ValueError("give angle_deg, step_um and pixel_um, or offsets")
        shift = shift_px(angle_deg, step_um, pixel_um)
        w0, b0 = plan(shape, shift=shift)
    else:
        w0, b0 = (None, None) if (origin is not None and width is not None) else plan(
            shape, offsets=offsets)
    origin = b0 if origin is None else int(origin)
    width = w0 if width is None else int(width)
    n, r, _ = shape
    out = dict(out or {})
    res = {"origin": origin, "width": width}
    for key, want, shp in (("vol", vol, (n, r, width)), ("psum", psum, (r, width)),
                           ("pmax", pmax, (r, width))):
        if not want:
            continue
        t = out.get(key)
        if t is None:
            t = torch.empty(shp, dtype=torch.float32, device=dev)
        elif t.shape != shp or t.dtype != torch.float32 or not t.is_contiguous() or t.device != dev:
            raise ValueError(f"out[{key!r}] must be contiguous float32 {shp} on {dev}")
        res[key] = t
    od = None if offsets is None else _offsets_dev(offsets, dev)
    res["_offsets_dev"] = od          # keep alive until the kernel has read it
    return shape, shift, w0, res


def _autotune_call(stack, shape, shift, res, reps, s):
    tn = L.Tune()
    ms = ctypes.c_double()
    st = L.lib().dsk_deskew_autotune(
        _vp(stack), int(stack.dtype == torch.float32), _dims(shape), _vp(res["_offsets_dev"]),
        float(shift or 0.0), res["origin"], _vp(res.get("vol")), _vp(res.get("psum")),
        _vp(res.get("pmax")), res["width"], int(reps), s, ctypes.byref(tn), ctypes.byref(ms))
    L.check(st, "dsk_deskew_autotune")
    return tn, ms.value


def autotune(stack: torch.Tensor, angle_deg=None, step_um=None, pixel_um=None, *,
             offsets=None, origin=None, width=None, vol=True, psum=True, pmax=True,
             out=None, reps=6, stream=None):
    """Launch shape for deskewing stacks of this frame on this device.

    Arguments as :func:`deskew`.  Times the library's candidate shapes
    (pacing rate, columns per lane) on this stack and returns
    ``{"tune": shape dict, "ms": mean time}``; the choice is
    remembered per frame (and in the ``DSK_TUNE_CACHE`` file when that
    variable is set), so later calls return at once.  Pass the shape as
    ``deskew(..., tune=...)``, or call ``deskew(..., tune="auto")``.
    """
    shape, shift, _, res = _setup(stack, angle_deg, step_um, pixel_um, offsets, origin, width,
                                  vol, psum, pmax, out)
    tn, ms = _autotune_call(stack, shape, shift, res, reps, _stream(stream))
    return {"tune": tn.as_dict(), "ms": ms}


def deskew(stack: torch.Tensor, angle_deg=None, step_um=None, pixel_um=None, *,
           offsets=None, origin=None, width=None, vol=True, psum=True, pmax=True,
           out=None, tune=None, stream=None):
    """Deskew ``stack`` and project it (one fused pass).

    Geometry is either (angle_deg, step_um, pixel_um) for a uniform scan, or
    explicit per-plane ``offsets`` in pixels.  ``origin``/``width`` default
    to the full frame.  ``out`` may hold preallocated ``vol``/``psum``/
    ``pmax`` tensors.  ``tune``: None (the library default), a launch-shape
    dict, or ``"auto"`` (the shape :func:`autotune` picks for this frame,
    measured on the first call).  Returns a dict with the outputs,
    ``origin`` and ``width``.
    """
    shape, shift, w0, res = _setup(stack, angle_deg, step_um, pixel_um, offsets, origin, width,
                                   vol, psum, pmax, out)
    origin, width, od = res["origin"], res["width"], res["_offsets_dev"]
    v, ps, pm = res.get("vol"), res.get("psum"), res.get("pmax")
    lib = L.lib()
    s = _stream(stream)
    if isinstance(tune, str):
        if tune != "auto":
            raise ValueError("tune must be None, a shape dict or 'auto'")
        tn = _autotune_call(stack, shape, shift, res, 6, s)[0]
    else:
        tn = _tune(tune)
    is_f32 = stack.dtype == torch.float32
    if od is None and tn is None and not is_f32 and width == w0:
        st = lib.dsk_deskew_u16(_vp(stack), _dims(shape), L.Geom(angle_deg, step_um, pixel_um),
                                _vp(v), _vp(ps), _vp(pm), 0, s)
        L.check(st, "dsk_deskew_u16")
        return res
    if tn is not None or od is None:
        st = lib.dsk_deskew_offsets_tuned(_vp(stack), int(is_f32), _dims(shape), _vp(od),
                                          float(shift or 0.0), origin, _vp(v), _vp(ps), _vp(pm),
                                          width, ctypes.byref(tn) if tn is not None else None, s)
        L.check(st, "dsk_deskew_offsets_tuned")
    elif is_f32:
        st = lib.dsk_deskew_offsets_f32(_vp(stack), _dims(shape), _vp(od), origin, _vp(v),
                                        _vp(ps), _vp(pm), width, s)
        L.check(st, "dsk_deskew_offsets_f32")
    else:
        st = lib.dsk_deskew_offsets_u16(_vp(stack), _dims(shape), _vp(od), origin, _vp(v),
                                        _vp(ps), _vp(pm), width, s)
        L.check(st, "dsk_deskew_offsets_u16")
    return res


def backward(stack, grad_vol, offsets_dev, origin, *, grad_in=True, grad_offsets=True,
             stream=None, noalloc=False):
    """Adjoint (grad wrt the float32 stack) and/or per-plane shear gradient.

    ``offsets_dev`` is a float64 CUDA tensor; ``grad_vol`` is float32
    [planes][rows][width].  Returns (grad_in or None, grad_offsets or None).
    ``noalloc`` calls the library's allocation-free variant (its partial
    sums in a library-owned device array; calls on one device must not
    overlap) instead of passing a workspace.
    """
    _check_stack(grad_vol, (torch.float32,))
    _check_stack(stack, (torch.float32,))
    n, r, w = grad_vol.shape
    if stack.shape[:2] != grad_vol.shape[:2]:
        raise ValueError("stack and grad_vol disagree in planes/rows")
    c = stack.shape[2]
    if offsets_dev.dtype != torch.float64 or not offsets_dev.is_cuda or offsets_dev.numel() != n:
        raise ValueError("offsets_dev must be a float64 CUDA tensor with one entry per plane")
    offsets_dev = offsets_dev.contiguous()
    dev = grad_vol.device
    dims = L.Dims(n, r, c)
    gi = torch.empty((n, r, c), dtype=torch.float32, device=dev) if grad_in else None
    go = torch.empty((n,), dtype=torch.float64, device=dev) if grad_offsets else None
    lib = L.lib()
    if noalloc:
        st = lib.dsk_backward_f32_noalloc(_vp(stack), _vp(grad_vol), dims, _vp(offsets_dev),
                                          int(origin), int(w), _vp(gi), _vp(go), _stream(stream))
        L.check(st, "dsk_backward_f32_noalloc")
        return gi, go
    ws = None
    wsb = 0
    if grad_offsets:
        wsb = int(lib.dsk_shear_grad_workspace_bytes(dims))
        ws = torch.empty((max(1, wsb // 8),), dtype=torch.float64, device=dev)
    st = lib.dsk_backward_f32(_vp(stack), _vp(grad_vol), dims, _vp(offsets_dev), int(origin),
                              int(w), _vp(gi), _vp(go), _vp(ws), wsb, _stream(stream))
    L.check(st, "dsk_backward_f32")
    return gi, go


def adjoint(grad_vol, offsets_dev, origin, cols, stream=None):
    """Transpose of the remap: grad_vol [N][R][W] -> [N][R][cols]."""
    _check_stack(grad_vol, (torch.float32,))
    n, r, w = grad_vol.shape
    dims = L.Dims(n, r, int(cols))
    gi = torch.empty((n, r, int(cols)), dtype=torch.float32, device=grad_vol.device)
    st = L.lib().dsk_deskew_adjoint_f32(_vp(grad_vol), dims, _vp(offsets_dev.contiguous()),
                                        int(origin), int(w), _vp(gi), _stream(stream))
    L.check(st, "dsk_deskew_adjoint_f32")
    return gi


def shear_grad(stack, grad_vol, offsets_dev, origin, stream=None):
    """Per-plane d(loss)/d(offset) in FP64 given d(loss)/dD."""
    _check_stack(stack, (torch.float32,))
    _check_stack(grad_vol, (torch.float32,))
    n, r, c = stack.shape
    w = grad_vol.shape[2]
    dims = L.Dims(n, r, c)
    lib = L.lib()
    wsb = int(lib.dsk_shear_grad_workspace_bytes(dims))
    ws = torch.empty((max(1, wsb // 8),), dtype=torch.float64, device=stack.device)
    go = torch.empty((n,), dtype=torch.float64, device=stack.device)
    st = lib.dsk_shear_grad_f32(_vp(stack), _vp(grad_vol), dims, _vp(offsets_dev.contiguous()),
                                int(origin), int(w), _vp(go), _vp(ws), wsb, _stream(stream))
    L.check(st, "dsk_shear_grad_f32")
    return go


def view_plan(shape, theta_deg, angle_deg, step_um, pixel_um):
    """Geometry of the shear-warp view at ``theta_deg`` from the optical axis
    (Fig. 3): dict with the per-image ``shear`` s' = z cos(theta) /
    (p cos(theta - alpha)), the column ``stretch`` cos(theta - alpha), the
    remap frame ``proj_width``/``origin`` and the view ``width``."""
    s, k = ctypes.c_double(), ctypes.c_double()
    w, b, vw = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = L.lib().dsk_view_plan(_dims(shape), L.Geom(angle_deg, step_um, pixel_um),
                               float(theta_deg), ctypes.byref(s), ctypes.byref(k),
                               ctypes.byref(w), ctypes.byref(b), ctypes.byref(vw))
    L.check(st, "dsk_view_plan")
    return {"shear": s.value, "stretch": k.value, "proj_width": int(w.value),
            "origin": int(b.value), "width": int(vw.value)}


def view(stack, theta_deg, angle_deg, step_um, pixel_um, *, vsum=True, vmax=True,
         width=None, workspace=None, stream=None):
    """Shear-warp view of a uint16 stack (Fig. 3): remap with the view's
    shift, project (sum and max) and stretch the projections along the
    column axis.  Returns a dict with ``vsum``/``vmax`` float32 [rows][width]
    and the geometry of :func:`view_plan`."""
    _check_stack(stack, (torch.uint16,))
    shape = tuple(stack.shape)
    g = view_plan(shape, theta_deg, angle_deg, step_um, pixel_um)
    if width is not None:
        g["width"] = int(width)
    dims = _dims(shape)
    lib = L.lib()
    need = int(lib.dsk_view_workspace_bytes(dims, g["proj_width"]))
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty((max(1, need // 4),), dtype=torch.float32, device=stack.device)
    r = shape[1]
    res = dict(g)
    for key, want in (("vsum", vsum), ("vmax", vmax)):
        if want:
            res[key] = torch.empty((r, g["width"]), dtype=torch.float32, device=stack.device)
    st = lib.dsk_view_u16(_vp(stack), dims, g["shear"], g["stretch"], g["origin"],
                          g["proj_width"], _vp(res.get("vsum")), _vp(res.get("vmax")),
                          g["width"], _vp(workspace), need, _stream(stream))
    L.check(st, "dsk_view_u16")
    res["_workspace"] = workspace
    return res


def stretch(proj, factor, width=None, stream=None):
    """Stretch every row of a float32 [rows][W] CUDA tensor along the column
    axis: column j samples the row at j / factor, linear, zero outside."""
    if not isinstance(proj, torch.Tensor) or proj.dim() != 2 or not proj.is_cuda or \
            proj.dtype != torch.float32 or not proj.is_contiguous():
        raise ValueError("proj must be a contiguous float32 CUDA tensor [rows][W]")
    rows, w_in = proj.shape
    if width is None:
        wout = ctypes.c_int64()
        L.check(L.lib().dsk_stretch_width(w_in, float(factor), ctypes.byref(wout)),
                "dsk_stretch_width")
        width = wout.value
    out = torch.empty((rows, int(width)), dtype=torch.float32, device=proj.device)
    st = L.lib().dsk_stretch_f32(_vp(proj), rows, w_in, float(factor), _vp(out), int(width),
                                 _stream(stream))
    L.check(st, "dsk_stretch_f32")
    return out


def deskew_channels(frames, col0s, cols, angle_deg, step_um, pixel_um, *, vol=True, psum=True,
                    pmax=True, streams=None):
    """Deskew the colour channels of multi-channel camera frames (each raw
    image split into its channels, every channel deskewed on its own),
    reading each channel in place.  ``frames``: contiguous uint16 CUDA
    tensor [planes][rows][frame_cols]; channel k is columns
    [col0s[k], col0s[k] + cols).  Channel k runs on ``streams[k]`` (default:
    one new stream per channel, joined back to the current stream).
    Returns one result dict per channel, as :func:`deskew`."""
    _check_stack(frames, (torch.uint16,))
    n, r, fc = (int(v) for v in frames.shape)
    cols = int(cols)
    dims = L.Dims(n, r, cols)
    geom = L.Geom(angle_deg, step_um, pixel_um)
    w, b = plan((n, r, cols), shift=shift_px(angle_deg, step_um, pixel_um))
    cur = torch.cuda.current_stream(frames.device)
    own = streams is None
    if own:
        streams = [torch.cuda.Stream(device=frames.device) for _ in col0s]
    lib = L.lib()
    out = []
    for k, c0 in enumerate(col0s):
        s = streams[k]
        if own:
            s.wait_stream(cur)
        res = {"origin": b, "width": w, "col0": int(c0)}
        with torch.cuda.stream(s):
            for key, want, shp in (("vol", vol, (n, r, w)), ("psum", psum, (r, w)),
                                   ("pmax", pmax, (r, w))):
                if want:
                    res[key] = torch.empty(shp, dtype=torch.float32, device=frames.device)
        st = lib.dsk_deskew_channel_u16(_vp(frames), fc, int(c0), dims, geom, _vp(res.get("vol")),
                                        _vp(res.get("psum")), _vp(res.get("pmax")), 0,
                                        ctypes.c_void_p(s.cuda_stream))
        L.check(st, "dsk_deskew_channel_u16")
        out.append(res)
    if own:
        for s in streams:
            cur.wait_stream(s)
        for res in out:
            for key in ("vol", "psum", "pmax"):
                if key in res:
                    res[key].record_stream(cur)
    return out


def affine_plan(shape, angle_deg, step_um, pixel_um, dy_um=None):
    """(Y0, ny) of the real-space grid with scan step ``dy_um`` (default: the
    pixel size)."""
    dy = float(pixel_um if dy_um is None else dy_um)
    y0, ny = ctypes.c_double(), ctypes.c_int64()
    st = L.lib().dsk_affine_plan(_dims(shape), L.Geom(angle_deg, step_um, pixel_um), dy,
                                 ctypes.byref(y0), ctypes.byref(ny))
    L.check(st, "dsk_affine_plan")
    return y0.value, int(ny.value)


def affine(stack, angle_deg, step_um, pixel_um, dy_um=None, *, y0=None, ny=None, out=None,
           stream=None):
    """Real-space (affine) deskew of a uint16 CUDA stack: float32
    [ny][rows][cols] on the Cartesian grid Y = Y0 + y dy, X = row,
    Z = column p sin(alpha).  Returns (vol, (Y0, ny))."""
    _check_stack(stack, (torch.uint16,))
    dy = float(pixel_um if dy_um is None else dy_um)
    y0_, ny_ = affine_plan(tuple(stack.shape), angle_deg, step_um, pixel_um, dy)
    y0 = y0_ if y0 is None else float(y0)
    ny = ny_ if ny is None else int(ny)
    n, r, c = (int(v) for v in stack.shape)
    if out is None:
        out = torch.empty((ny, r, c), dtype=torch.float32, device=stack.device)
    elif tuple(out.shape) != (ny, r, c) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError(f"out must be contiguous float32 {(ny, r, c)}")
    st = L.lib().dsk_affine_u16(_vp(stack), _dims(stack.shape),
                                L.Geom(angle_deg, step_um, pixel_um), dy, y0, ny, _vp(out),
                                _stream(stream))
    L.check(st, "dsk_affine_u16")
    return out, (y0, ny)
