"""Rolling display mode: the projections refreshed after every camera image
(the paper's rolling update for slow acquisitions, Fig. 4a), one kernel per
image.  Device state: the current deskewed images, a max-tree over them and
an FP64 running sum (see ``dsk_rolling_update_u16`` in include/deskew.h).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from . import api


class RollingView:
    """Live projections of a stack whose images arrive one at a time.

    ``planes, rows, cols``: stack shape; geometry as (angle_deg, step_um,
    pixel_um), or the per-image shift in pixels (``shift_px``).  ``update(n, image)`` writes raw image n ([rows][cols] uint16
    CUDA tensor) and refreshes ``psum``/``pmax``; ``vol`` holds the current
    deskewed images.
    """

    def __init__(self, planes, rows, cols, angle_deg=None, step_um=None, pixel_um=None,
                 device="cuda", shift_px=None):
        self.dims = L.Dims(int(planes), int(rows), int(cols))
        self.shift = (float(shift_px) if shift_px is not None
                      else api.shift_px(angle_deg, step_um, pixel_um))
        self.width, self.origin = api.plan((planes, rows, cols), shift=self.shift)
        w = self.width
        self.vol = torch.empty((planes, rows, w), dtype=torch.float32, device=device)
        tb = int(L.lib().dsk_rolling_tree_bytes(self.dims, w))
        self.tree = torch.empty(max(1, tb // 4), dtype=torch.float32, device=device)
        self.sum64 = torch.empty((rows, w), dtype=torch.float64, device=device)
        self.psum = torch.empty((rows, w), dtype=torch.float32, device=device)
        self.pmax = torch.empty((rows, w), dtype=torch.float32, device=device)
        self.reset()

    def reset(self, stream=None):
        st = L.lib().dsk_rolling_reset(self.dims, self.width, api._vp(self.vol),
                                       api._vp(self.tree), api._vp(self.sum64),
                                       api._vp(self.psum), api._vp(self.pmax),
                                       api._stream(stream))
        L.check(st, "dsk_rolling_reset")

    def update(self, n: int, image: torch.Tensor, stream=None):
        if image.dtype != torch.uint16 or not image.is_cuda or not image.is_contiguous():
            raise ValueError("image must be a contiguous uint16 CUDA tensor")
        if tuple(image.shape) != (self.dims.rows, self.dims.cols):
            raise ValueError(f"image must be [{self.dims.rows}][{self.dims.cols}]")
        st = L.lib().dsk_rolling_update_u16(api._vp(image), int(n), self.dims, None, self.shift,
                                            self.origin, self.width, api._vp(self.vol),
                                            api._vp(self.tree), api._vp(self.sum64),
                                            api._vp(self.psum), api._vp(self.pmax),
                                            api._stream(stream))
        L.check(st, "dsk_rolling_update_u16")
