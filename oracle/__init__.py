"""CPU FP64 oracle for the r1-sparse block Jacobian, its block-Jacobi
preconditioner and restarted GMRES.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg call it.  It
shares no code with the HIP path: it reads the same generated input arrays
and computes everything again from the definitions, slowly and plainly, in
float64.

Modules (each function cites the passage it follows):
  mesh        structured-mesh adjacency (first-order FV stencil, section 3)
  assemble    dense-block (BSR) assembly of J = S + sum_blocks u v^T
  ops         BSR matvec and transpose, full dense J for tiny meshes
  formats     CSR, r1-sparse, BSR and BR1-BSR formats of section 5.1 and the
              structured (CSR + block rank-one) matvec of section 5.2
  blockjacobi dense LU block-Jacobi and the Sherman-Morrison-Woodbury local
              solve of section 6
  gmres       restarted right-preconditioned GMRES (section 6, right
              preconditioning)
  grads       gradients of a linear loss through x = J^{-1} b
  storage     stored-value counts of both representations (section 3,
              "Jacobian Complexity")

Pins (tests marked "not gpu") tie every function to something other than
itself: the paper's worked examples, library routines on special cases,
brute-force dense solves and closed forms.  Mixed-precision iteration counts
and timings have no such pin: parity unpinned.
"""
