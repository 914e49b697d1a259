"""MI355X (gfx950) constrained-Gaussian-realization fill-in of masked flat-sky maps.

Hot path of Bucher & Louis (arXiv:1109.0286), Sec. 2-3: unconstrained
Gaussian realization + preconditioned CG solve for the masked pixels, every
operator apply a hand-written HIP 2D FFT / spectral multiply / mask pass.
The package is a thin binding of libfill.so (C ABI, include/fill.h).
"""

from .fill import *  # noqa: F401,F403
from .fill import Plan, BatchPlan, Group, Strips, realize_multi, philox_words, EXPORTS, LIB_PATH  # noqa: F401


def autograd_fill():
    """The torch.autograd.Function over the fill (imported on demand)."""
    from .autograd import FillFn
    return FillFn
