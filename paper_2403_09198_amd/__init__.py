"""r1-sparse block Jacobian, SMW block-Jacobi and GMRES on MI355X (gfx950).

The compute runs in hand-written HIP kernels behind the C ABI declared in
include/r1s.h (libr1s.so, built in-tree).  The shared library is loaded on
first use; nothing here falls back to a CPU implementation.
"""
__all__ = ["gen"]
