"""ctypes binding of libdeskew.so (the C ABI declared in include/deskew.h).

Argument marshalling only: every step of the deskew runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built;
there is no fallback implementation.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# DSK_LIB may name another build of the same library (the host-ASan build)
LIB_PATH = os.environ.get("DSK_LIB") or os.path.join(_PKG, "libdeskew.so")

c_i32, c_i64, c_dbl, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_size_t)

DSK_OK, DSK_EINVAL, DSK_ESHAPE, DSK_EHIP, DSK_ENOMEM, DSK_EBUDGET = 0, -1, -2, -3, -4, -5


class Dims(ctypes.Structure):
    _fields_ = [("planes", c_i32), ("rows", c_i32), ("cols", c_i32)]


class Geom(ctypes.Structure):
    _fields_ = [("angle_deg", c_dbl), ("step_um", c_dbl), ("pixel_um", c_dbl)]


class Tune(ctypes.Structure):
    _fields_ = [("block", c_i32), ("per_thread", c_i32), ("nt_store", c_i32),
                ("unroll", c_i32), ("wg_per_cu", c_i32), ("pace_gbs", c_i32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Job(ctypes.Structure):
    _fields_ = [("in_", c_vp), ("dims", Dims), ("offsets_dev", c_vp),
                ("shift_px", c_dbl), ("origin", c_i64), ("out_width", c_i64),
                ("vol", c_vp), ("psum", c_vp), ("pmax", c_vp)]


class DeskewError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_SIGS = {
    "dsk_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dsk_debug_bounds_violations": (ctypes.c_int, [ctypes.POINTER(ctypes.c_ulonglong),
                                                   ctypes.c_int]),
    "dsk_shift_px": (ctypes.c_int, [Geom, ctypes.POINTER(c_dbl)]),
    "dsk_plan": (ctypes.c_int, [Dims, c_vp, c_dbl, ctypes.POINTER(c_i64),
                                ctypes.POINTER(c_i64)]),
    "dsk_deskew_u16": (ctypes.c_int, [c_vp, Dims, Geom, c_vp, c_vp, c_vp, c_i64, c_vp]),
    "dsk_deskew_channel_u16": (ctypes.c_int, [c_vp, c_i64, c_i64, Dims, Geom, c_vp, c_vp, c_vp,
                                              c_i64, c_vp]),
    "dsk_deskew_offsets_u16": (ctypes.c_int, [c_vp, Dims, c_vp, c_i64, c_vp, c_vp, c_vp,
                                              c_i64, c_vp]),
    "dsk_deskew_offsets_f32": (ctypes.c_int, [c_vp, Dims, c_vp, c_i64, c_vp, c_vp, c_vp,
                                              c_i64, c_vp]),
    "dsk_deskew_offsets_tuned": (ctypes.c_int, [c_vp, ctypes.c_int, Dims, c_vp, c_dbl, c_i64,
                                                c_vp, c_vp, c_vp, c_i64,
                                                ctypes.POINTER(Tune), c_vp]),
    "dsk_deskew_autotune": (ctypes.c_int, [c_vp, ctypes.c_int, Dims, c_vp, c_dbl, c_i64,
                                           c_vp, c_vp, c_vp, c_i64, ctypes.c_int, c_vp,
                                           ctypes.POINTER(Tune), ctypes.POINTER(c_dbl)]),
    "dsk_deskew_adjoint_f32": (ctypes.c_int, [c_vp, Dims, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "dsk_shear_grad_workspace_bytes": (c_sz, [Dims]),
    "dsk_shear_grad_f32": (ctypes.c_int, [c_vp, c_vp, Dims, c_vp, c_i64, c_i64, c_vp, c_vp,
                                          c_sz, c_vp]),
    "dsk_backward_f32": (ctypes.c_int, [c_vp, c_vp, Dims, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp,
                                        c_sz, c_vp]),
    "dsk_backward_f32_noalloc": (ctypes.c_int, [c_vp, c_vp, Dims, c_vp, c_i64, c_i64, c_vp,
                                                c_vp, c_vp]),
    "dsk_batch_create": (ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_int,
                                        ctypes.POINTER(Tune), c_vp, ctypes.POINTER(c_vp)]),
    "dsk_batch_launch": (ctypes.c_int, [c_vp, c_vp]),
    "dsk_batch_launch_direct": (ctypes.c_int, [c_vp, c_vp]),
    "dsk_batch_get_tune": (ctypes.c_int, [c_vp, ctypes.POINTER(Tune), ctypes.POINTER(c_dbl)]),
    "dsk_batch_get_mode": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_int)]),
    "dsk_batch_destroy": (ctypes.c_int, [c_vp]),
    "dsk_jobs_table_bytes": (c_sz, [ctypes.c_int]),
    "dsk_rolling_tree_bytes": (c_sz, [Dims, c_i64]),
    "dsk_rolling_reset": (ctypes.c_int, [Dims, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "dsk_rolling_update_u16": (ctypes.c_int, [c_vp, c_i32, Dims, c_vp, c_dbl, c_i64, c_i64,
                                              c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "dsk_jobs_launch": (ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_int, c_vp, c_vp, c_sz,
                                       ctypes.POINTER(Tune), c_vp]),
    "dsk_view_plan": (ctypes.c_int, [Dims, Geom, c_dbl, ctypes.POINTER(c_dbl),
                                     ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64),
                                     ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "dsk_view_workspace_bytes": (c_sz, [Dims, c_i64]),
    "dsk_view_u16": (ctypes.c_int, [c_vp, Dims, c_dbl, c_dbl, c_i64, c_i64, c_vp, c_vp, c_i64,
                                    c_vp, c_sz, c_vp]),
    "dsk_stretch_width": (ctypes.c_int, [c_i64, c_dbl, ctypes.POINTER(c_i64)]),
    "dsk_stretch_f32": (ctypes.c_int, [c_vp, c_i64, c_i64, c_dbl, c_vp, c_i64, c_vp]),
    "dsk_affine_plan": (ctypes.c_int, [Dims, Geom, c_dbl, ctypes.POINTER(c_dbl),
                                       ctypes.POINTER(c_i64)]),
    "dsk_affine_u16": (ctypes.c_int, [c_vp, Dims, Geom, c_dbl, c_dbl, c_i64, c_vp, c_vp]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2211_00645_amd.build` "
                "(the deskew has no non-HIP implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().dsk_status_string(int(status)).decode()


def check(status: int, where: str):
    if status != DSK_OK:
        raise DeskewError(status, where)
