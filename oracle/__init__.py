"""Plain FP64 CPU oracle for the wavelet multilevel l1 deblurring method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package.  It
shares no code with the GPU library and imports nothing from it; the product
path never calls it.

Everything here is written from the paper's definitions, in float64, with no
blocking or fusion: slow and obviously correct.  Images are 2-D arrays X[i, j]
(i = row, j = column); the paper's vector x = vec(X) stacks columns
(column-major), so ``vec`` / ``unvec`` below convert at the boundary.

Parity status of each part (what pins it) is listed in the module docstrings.
One result is "parity unpinned": the end-to-end reconstructions against the
paper's own figures and tables, which need the paper's images and MATLAB.
"""
from . import operators, hierarchy, krylov, gcv, solvers, vcycle, objective, metrics

__all__ = ["operators", "hierarchy", "krylov", "gcv", "solvers", "vcycle", "objective",
           "metrics"]
