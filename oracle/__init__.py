"""FP64 CPU oracle for the deskew + projection path (arXiv 2211.00645).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product package never does.
It wraps ``liboracle.so`` (plain C, built by ``oracle/build.py``), which shares
no source with the HIP library.

Every function here follows the paper's definitions, cited per function:
  * ``shift_px``   -- Eq. 1 (``l = z cos(alpha)``), converted to pixels.
  * ``frame``      -- the larger image each raw image is remapped into
                      ("Physical principles", remap paragraph; Fig. 2c).
  * ``deskew``     -- the remap with linear interpolation, plus the maximum
                      projection (Fig. 2d) and the sum projection.
  * ``adjoint``    -- transpose of the remap, as an explicit scatter.
  * ``shear_grad`` -- derivative of a loss with respect to each image offset.
  * ``view_geometry``, ``warp``, ``view`` -- the shear-warp rotated view
                      (Fig. 3): projection of the stack remapped with a
                      changed shift, stretched along the column axis.
  * ``affine_frame``, ``affine`` -- the real-space (affine) deskew the paper
                      contrasts the remap with: the stack resampled onto a
                      Cartesian grid by interpolation between images.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_threads.argtypes = []
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_shift_px.restype = ctypes.c_double
    lib.orc_shift_px.argtypes = [ctypes.c_double] * 3
    lib.orc_offsets_uniform.restype = None
    lib.orc_offsets_uniform.argtypes = [_i64, ctypes.c_double, _dp]
    lib.orc_frame.restype = None
    lib.orc_frame.argtypes = [_i64, _dp, _i64, ctypes.POINTER(_i64),
                              ctypes.POINTER(_i64)]
    lib.orc_deskew.restype = None
    lib.orc_deskew.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64, _i64, _i64,
                               _dp, _i64, _i64, _i64, _i64,
                               _fp, _dp, _fp, _fp]
    lib.orc_adjoint.restype = None
    lib.orc_adjoint.argtypes = [_fp, _i64, _i64, _i64, _dp, _i64, _i64,
                                _fp, _dp]
    lib.orc_shear_grad.restype = None
    lib.orc_shear_grad.argtypes = [_fp, _fp, _i64, _i64, _i64, _dp, _i64,
                                   _i64, _dp]
    lib.orc_view_geometry.restype = None
    lib.orc_view_geometry.argtypes = [ctypes.c_double] * 4 + [_dp, _dp]
    lib.orc_view_width.restype = _i64
    lib.orc_view_width.argtypes = [_i64, ctypes.c_double]
    lib.orc_warp.restype = None
    lib.orc_warp.argtypes = [_dp, _i64, _i64, ctypes.c_double, _i64, _dp]
    lib.orc_affine_frame.restype = None
    lib.orc_affine_frame.argtypes = [_i64, _i64] + [ctypes.c_double] * 4 + [_dp,
                                                                            ctypes.POINTER(_i64)]
    lib.orc_affine.restype = None
    lib.orc_affine.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64, _i64, _i64] + \
        [ctypes.c_double] * 5 + [_i64, _fp, _dp]
    _lib = lib
    return lib


def _ptr(a, typ):
    if a is None:
        return None
    return a.ctypes.data_as(typ)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP threads of the oracle's parallel loops (timing only)."""
    _load().orc_set_threads(int(n))


def shift_px(angle_deg: float, step_um: float, pixel_um: float) -> float:
    """Per-image lateral shift in pixels, Eq. 1: (z cos(alpha)) / p."""
    return _load().orc_shift_px(float(angle_deg), float(step_um), float(pixel_um))


def offsets_uniform(n_planes: int, shift: float) -> np.ndarray:
    """o[n] = n * s for a uniform scan (Eq. 1 accumulated n times)."""
    out = np.empty(n_planes, np.float64)
    _load().orc_offsets_uniform(n_planes, float(shift), _ptr(out, _dp))
    return out


def frame(offsets, cols: int):
    """(origin b, width W) of the larger image holding every shifted image."""
    o = np.ascontiguousarray(offsets, np.float64)
    b, w = _i64(), _i64()
    _load().orc_frame(o.size, _ptr(o, _dp), int(cols), ctypes.byref(b),
                      ctypes.byref(w))
    return int(b.value), int(w.value)


def deskew(stack, offsets, origin=None, width=None, rows=None, vol=True,
           vol64=False):
    """Remap every image of ``stack`` [N][R][C] (uint16 or float32) to its
    offset and project over the image axis.

    Returns a dict with ``vol`` (float32 [N][nr][W]) if ``vol``, ``vol64``
    (float64) if ``vol64``, and ``psum``/``pmax`` (float32 [nr][W]) for the
    row range ``rows=(r0, r1)`` (default: all rows).
    """
    s = np.ascontiguousarray(stack)
    if s.dtype == np.uint16:
        is_f32 = 0
    elif s.dtype == np.float32:
        is_f32 = 1
    else:
        raise TypeError("oracle deskew takes uint16 or float32 stacks")
    n, r, c = s.shape
    o = np.ascontiguousarray(offsets, np.float64)
    assert o.shape == (n,)
    if origin is None or width is None:
        b0, w0 = frame(o, c)
        origin = b0 if origin is None else origin
        width = w0 if width is None else width
    r0, r1 = (0, r) if rows is None else rows
    nr = r1 - r0
    out = {"origin": int(origin), "width": int(width)}
    v = np.empty((n, nr, width), np.float32) if vol else None
    v64 = np.empty((n, nr, width), np.float64) if vol64 else None
    ps = np.empty((nr, width), np.float32)
    pm = np.empty((nr, width), np.float32)
    _load().orc_deskew(s.ctypes.data_as(ctypes.c_void_p), is_f32, n, r, c,
                       _ptr(o, _dp), int(origin), int(width), int(r0), int(r1),
                       _ptr(v, _fp), _ptr(v64, _dp), _ptr(ps, _fp),
                       _ptr(pm, _fp))
    if vol:
        out["vol"] = v
    if vol64:
        out["vol64"] = v64
    out["psum"] = ps
    out["pmax"] = pm
    return out


def adjoint(grad_vol, offsets, origin, cols, as_f64=False):
    """Transpose of the remap applied to ``grad_vol`` [N][R][W] -> [N][R][C]."""
    g = np.ascontiguousarray(grad_vol, np.float32)
    n, r, w = g.shape
    o = np.ascontiguousarray(offsets, np.float64)
    out32 = None if as_f64 else np.empty((n, r, cols), np.float32)
    out64 = np.empty((n, r, cols), np.float64) if as_f64 else None
    _load().orc_adjoint(_ptr(g, _fp), n, r, int(cols), _ptr(o, _dp),
                        int(origin), w, _ptr(out32, _fp), _ptr(out64, _dp))
    return out64 if as_f64 else out32


def shear_grad(stack, grad_vol, offsets, origin):
    """d(loss)/d(o[n]) for every image n, FP64, given d(loss)/dD."""
    s = np.ascontiguousarray(stack, np.float32)
    g = np.ascontiguousarray(grad_vol, np.float32)
    n, r, c = s.shape
    w = g.shape[2]
    assert g.shape[:2] == (n, r)
    o = np.ascontiguousarray(offsets, np.float64)
    out = np.empty(n, np.float64)
    _load().orc_shear_grad(_ptr(s, _fp), _ptr(g, _fp), n, r, c, _ptr(o, _dp),
                           int(origin), w, _ptr(out, _dp))
    return out


def view_geometry(theta_deg, angle_deg, step_um, pixel_um):
    """(shift per image s', stretch factor) of the view at ``theta_deg`` from
    the optical axis: s' = z cos(theta) / (p cos(theta - alpha)), stretch
    cos(theta - alpha) (Fig. 3)."""
    s, w = ctypes.c_double(), ctypes.c_double()
    _load().orc_view_geometry(float(theta_deg), float(angle_deg), float(step_um),
                              float(pixel_um), ctypes.byref(s), ctypes.byref(w))
    return s.value, w.value


def view_width(width_in, warp_factor):
    """View columns whose source coordinate j / warp lies in the projection."""
    return int(_load().orc_view_width(int(width_in), float(warp_factor)))


def warp(proj, warp_factor, width_out=None):
    """Stretch every row of ``proj`` [R][W] along the column axis: view
    column j is the linear interpolation of the row at j / warp (zero
    outside).  FP64 in and out."""
    p = np.ascontiguousarray(proj, np.float64)
    rows, w_in = p.shape
    if width_out is None:
        width_out = view_width(w_in, warp_factor)
    out = np.empty((rows, width_out), np.float64)
    _load().orc_warp(_ptr(p, _dp), rows, w_in, float(warp_factor), int(width_out),
                     _ptr(out, _dp))
    return out


def view(stack, theta_deg, angle_deg, step_um, pixel_um, width_out=None):
    """Shear-warp view (Fig. 3): remap with the view's shift s', project over
    the image axis, stretch the projections by the view's factor.  Returns a
    dict with ``psum``/``pmax`` (FP64 [R][width_out]) and the geometry."""
    n, r, c = np.shape(stack)
    s, wf = view_geometry(theta_deg, angle_deg, step_um, pixel_um)
    offs = offsets_uniform(n, s)
    b, w_in = frame(offs, c)
    d = deskew(stack, offs, b, w_in, vol=False)
    if width_out is None:
        width_out = view_width(w_in, wf)
    return {"shear": s, "warp": wf, "origin": b, "proj_width": w_in,
            "width": int(width_out),
            "psum": warp(d["psum"], wf, width_out), "pmax": warp(d["pmax"], wf, width_out)}


def affine_frame(n_planes, cols, angle_deg, step_um, pixel_um, dy_um):
    """(Y0, ny) of the real-space grid: smallest scan coordinate of the
    stack's corners and the number of Y steps of ``dy_um`` covering it."""
    y0, ny = ctypes.c_double(), _i64()
    _load().orc_affine_frame(int(n_planes), int(cols), float(angle_deg), float(step_um),
                             float(pixel_um), float(dy_um), ctypes.byref(y0), ctypes.byref(ny))
    return y0.value, int(ny.value)


def affine(stack, angle_deg, step_um, pixel_um, dy_um, y0=None, ny=None, vol64=False):
    """Real-space deskew: vol[y][x][z] is the linear interpolation between
    images floor(u) and floor(u)+1 at raw column z, row x, with
    u = (Y0 + y dy - z p cos(alpha)) / z_step.  Returns float32 (or float64)
    [ny][rows][cols] and (Y0, ny)."""
    s = np.ascontiguousarray(stack)
    if s.dtype == np.uint16:
        is_f32 = 0
    elif s.dtype == np.float32:
        is_f32 = 1
    else:
        raise TypeError("oracle affine takes uint16 or float32 stacks")
    n, r, c = s.shape
    if y0 is None or ny is None:
        y0_, ny_ = affine_frame(n, c, angle_deg, step_um, pixel_um, dy_um)
        y0 = y0_ if y0 is None else y0
        ny = ny_ if ny is None else ny
    out32 = None if vol64 else np.empty((ny, r, c), np.float32)
    out64 = np.empty((ny, r, c), np.float64) if vol64 else None
    _load().orc_affine(s.ctypes.data_as(ctypes.c_void_p), is_f32, n, r, c, float(angle_deg),
                       float(step_um), float(pixel_um), float(dy_um), float(y0), int(ny),
                       _ptr(out32, _fp), _ptr(out64, _dp))
    return (out64 if vol64 else out32), (float(y0), int(ny))
