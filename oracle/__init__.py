"""FP64 CPU oracle for the w-stacking imager.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or call anything here; the imaging
library (HIP kernels behind the C ABI and its Python binding) shares no code
with it and never calls it.

Two parts:
  * ``wstack`` (O-WS): the reference w-stacking algorithm, step by step, in
    float64 (gridding loop in plain C, plane transforms with numpy's FFT or,
    at sampled pixels, the same sum as matrix products).
  * ``dft`` (O-DFT): the direct adjoint of the measurement equation with the
    exact w-term.
Both are pinned by tests against closed forms, invariants and brute force.

Parity unpinned: the absolute flux scale of the paper's own code, which rescales
uvw and whose flux differs from other imagers by its authors' account; this
oracle works in physical units instead.
"""

from . import kb, wstack, dft  # noqa: F401
from .wstack import (Params, prepare, wstack_image, wstack_predict, grid_stack, grid_plane, plane_transform,  # noqa: F401
                     direction_cosines)
from .dft import dft_image  # noqa: F401
from ._native import build  # noqa: F401
