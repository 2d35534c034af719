"""MI355X-native multi-level constrained-realization solver.

Hot path of Seljebotn et al. (2013): applying A = S^-1 + B Y^T N^-1 Y B and
its level operators on HEALPix RING grids with hand-written gfx950 HIP
kernels behind a C ABI (include/mlcr.h).  This package is a thin binding:
torch supplies device memory and streams, every step runs in libmlcr.so.
"""
from ._lib import MLCRError, load as load_library  # noqa: F401
from .api import (BF16X3, FP32, FP64, Geometry, KernelTimer, Ladder, Operator, Solver,  # noqa: F401
                  apply_A, apply_A_grouped, solve_grouped, cr_rhs, prior_band_grad,
                  cycle_counts, ladder_plan, nest2ring, sht_adjoint, sht_synth, tile_graph)

from . import autograd  # noqa: F401,E402
from . import autotune  # noqa: F401,E402

__all__ = ["autograd", "autotune", "MLCRError", "load_library", "BF16X3", "FP32", "FP64", "Geometry", "Operator",
           "apply_A", "apply_A_grouped", "solve_grouped", "cr_rhs", "sht_adjoint", "sht_synth", "KernelTimer",
           "Solver", "Ladder", "prior_band_grad", "nest2ring", "tile_graph",
           "ladder_plan", "cycle_counts"]
