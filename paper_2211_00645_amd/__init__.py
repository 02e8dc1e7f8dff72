"""MI355X-native deskew of oblique-plane light-sheet stacks (arXiv 2211.00645).

The hot path -- remap of every raw image to its lateral offset (Eq. 1) with
fused sum and maximum projections, its adjoint and shear gradient, ragged
batches, the live serving loop, the rolling update, shear-warp rotated
views, multi-channel frames and the real-space (affine) deskew -- runs in the HIP kernels of
``libdeskew.so`` (C ABI in ``include/deskew.h``).  Import is light: the
library is loaded on first use and its absence is an error, never a fallback.
"""
from .api import (adjoint, affine, affine_plan, autotune, backward, deskew,  # noqa: F401
                  deskew_channels, plan, shear_grad, shift_px, stretch, view, view_plan)

__all__ = ["deskew", "autotune", "deskew_channels", "plan", "shift_px", "backward", "adjoint",
           "shear_grad", "view", "view_plan", "stretch", "affine", "affine_plan"]
