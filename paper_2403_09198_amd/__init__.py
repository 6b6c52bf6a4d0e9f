"""r1-sparse block Jacobian, SMW block-Jacobi and GMRES on MI355X (gfx950).

The compute runs in hand-written HIP kernels behind the C ABI declared in
include/r1s.h (libr1s.so, built in-tree by `python -m
paper_2403_09198_amd.csrc.build`).  The shared library is loaded on first
use and nothing falls back to a CPU implementation.

  gen        seeded synthetic problems (shared input, no method arithmetic)
  r1s        binding of the C calls + R1Matrix / SMWPreconditioner /
             BSRMatrix / DenseLUPreconditioner / gmres / grad
  autograd   R1SolveFn: differentiable x = J^{-1} b
"""
__all__ = ["gen", "r1s", "autograd"]
