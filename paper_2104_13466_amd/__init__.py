"""libsdme: MI355X-native (gfx950) SDME high-order FEM hot path -- neo-Hookean
internal force and tangent action on tensor-product hexahedra with the SDME 1D
bases of arXiv 2104.13466, plus Jacobi-PCG, Newton, Newmark and central
difference drivers.  The compute path is the C-ABI library libsdme.so
(hand-written HIP kernels); this package is a thin binding over it."""
from . import sdme  # noqa: F401
from .sdme import (Context, SdmeError, basis_build, basis_eval, FP32, FP64, NODAL, MODAL,  # noqa: F401
                   SDME_M, SDME_K, SDME_H, MASK_BC, CHECK_JAC)
