"""Block-Jacobi preconditioning (section 6).

The preconditioner M is the inverse of the block-diagonal part of J.  Its
classical form (section 6) factors every diagonal block with a local LU; here
that is Doolittle elimination with partial pivoting, written out and
vectorised across blocks.

Section 6 also gives the variation this library accelerates: with the
diagonal block written as A_k = A_k^0 + U_k V_k^T (eq. R1_Block_Jacobian), its
inverse follows from the Sherman-Morrison-Woodbury identity (eq. SMW).  The
identity as printed adds the correction term; the correct identity (Golub &
Van Loan; Hager's review, which the paper cites) subtracts it:

    A^{-1} = A0^{-1} - A0^{-1} U C^{-1} V^T A0^{-1},  C = I + V^T A0^{-1} U,

and correspondingly the final assembly step is x = x0 - W z.  `smw_solve`
uses that sign; a test shows the printed sign fails to invert the block.
"""
import numpy as np

from . import assemble, mesh


class SingularBlock(ArithmeticError):
    pass


# ------------------------------------------------------------ dense LU ------
def lu_factor(A):
    """LU with partial pivoting of a stack of square blocks A [nb][m][m].

    Returns (LU, piv): LU holds the unit-lower multipliers below the diagonal
    and U on and above it; piv[:, k] is the row swapped with row k at step k.
    """
    LU = np.array(A, dtype=np.float64, copy=True)
    nb, m, _ = LU.shape
    piv = np.zeros((nb, m), dtype=np.int64)
    blk = np.arange(nb)
    for k in range(m):
        p = k + np.argmax(np.abs(LU[:, k:, k]), axis=1)
        piv[:, k] = p
        row_k = LU[blk, k, :].copy()
        LU[blk, k, :] = LU[blk, p, :]
        LU[blk, p, :] = row_k
        pivot = LU[:, k, k]
        if np.any(pivot == 0.0):
            raise SingularBlock(f"zero pivot in block {int(np.argmax(pivot == 0.0))}")
        LU[:, k + 1:, k] /= pivot[:, None]
        LU[:, k + 1:, k + 1:] -= LU[:, k + 1:, k, None] * LU[:, k, None, k + 1:]
    return LU, piv


def lu_solve(LU, piv, b):
    """Solve A x = b for every block; b has shape [nb][m] (or [nrhs][nb][m])."""
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 3:
        return np.stack([lu_solve(LU, piv, bi) for bi in b])
    x = b.copy()
    nb, m = x.shape
    blk = np.arange(nb)
    for k in range(m):  # apply the row swaps in order
        p = piv[:, k]
        tmp = x[blk, k].copy()
        x[blk, k] = x[blk, p]
        x[blk, p] = tmp
    for k in range(m):  # forward substitution, unit lower triangle
        x[:, k] -= np.einsum("bj,bj->b", LU[:, k, :k], x[:, :k])
    for k in range(m - 1, -1, -1):  # back substitution
        x[:, k] -= np.einsum("bj,bj->b", LU[:, k, k + 1:], x[:, k + 1:])
        x[:, k] /= LU[:, k, k]
    return x


def lu_solve_T(LU, piv, b):
    """Solve A^T x = b for every block.  With P A = L U, A^T = U^T L^T P, so
    solve U^T y = b, then L^T z = y, then undo the swaps in reverse order."""
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 3:
        return np.stack([lu_solve_T(LU, piv, bi) for bi in b])
    x = b.copy()
    nb, m = x.shape
    blk = np.arange(nb)
    for k in range(m):  # U^T is lower triangular
        x[:, k] -= np.einsum("bj,bj->b", LU[:, :k, k], x[:, :k])
        x[:, k] /= LU[:, k, k]
    for k in range(m - 1, -1, -1):  # L^T is unit upper triangular
        x[:, k] -= np.einsum("bj,bj->b", LU[:, k + 1:, k], x[:, k + 1:])
    for k in range(m - 1, -1, -1):
        p = piv[:, k]
        tmp = x[blk, k].copy()
        x[blk, k] = x[blk, p]
        x[blk, p] = tmp
    return x


# ------------------------------------------------------------- SMW form -----
def tridiag_solve(diag, sub, sup, r):
    """Solve a tridiagonal system (no pivoting) by LU of the band, i.e. the
    Thomas algorithm: d_0 = a_0, l_k = b_{k-1}/d_{k-1}, d_k = a_k - l_k c_{k-1};
    forward y_k = r_k - l_k y_{k-1}; backward x_k = (y_k - c_k x_{k+1}) / d_k.
    diag [n], sub[k] = T[k+1,k], sup[k] = T[k,k+1] (length n-1)."""
    n = len(diag)
    d = np.zeros(n)
    l = np.zeros(n)
    d[0] = diag[0]
    for k in range(1, n):
        l[k] = sub[k - 1] / d[k - 1]
        d[k] = diag[k] - l[k] * sup[k - 1]
    y = np.array(r, dtype=np.float64, copy=True)
    for k in range(1, n):
        y[k] -= l[k] * y[k - 1]
    x = np.zeros(n)
    x[n - 1] = y[n - 1] / d[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = (y[k] - sup[k] * x[k + 1]) / d[k]
    return x


def sparse_diag_solve(p, c, L, r):
    """x = (S_{c,C})^{-1} r.  Tridiagonal band without coupling: the level
    band and the 3 x 3 flow corner are uncoupled, so solve each on its own.
    A wider band or level/flow coupling: LAPACK's dense solve of the
    assembled sparse block."""
    r = np.asarray(r, dtype=np.float64)
    if mesh.pattern(p) != (1, 0):
        return np.linalg.solve(assemble.diagonal_sparse_block(p, c, L), r)
    x = np.zeros(L + 3)
    x[:L] = tridiag_solve(p["s_diag"][c, :L], p["s_sub"][c], p["s_sup"][c], r[:L])
    F = np.diag(p["s_diag"][c, L:])
    pairs = ((0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1))
    for t, (i, j) in enumerate(pairs):
        F[i, j] = p["s_flow"][c, t]
    x[L:] = np.linalg.solve(F, r[L:])
    return x


def smw_solve(p, c, L, r, sign=-1.0):
    """Solve D_{c,C} x = r with D = A0 + U V^T (eq. R1_Block_Jacobian) by the
    three SMW steps of section 6: (SMW-1) x0 = A0^{-1} r and W = A0^{-1} U;
    (SMW-2) C z = V^T x0 with C = I + V^T W; assemble x = x0 + sign * W z.
    sign = -1 is the correct identity; sign = +1 reproduces the printed one."""
    a, cnt = mesh.pair_range(p, 2)
    U = p["u"][c, a:a + cnt].T  # m x r
    V = p["v"][c, a:a + cnt].T
    x0 = sparse_diag_solve(p, c, L, r)
    W = np.column_stack([sparse_diag_solve(p, c, L, U[:, i]) for i in range(cnt)])
    Cm = np.eye(cnt) + V.T @ W
    z = np.linalg.solve(Cm, V.T @ x0)
    return x0 + sign * (W @ z)


def smw_inverse(p, c, L, sign=-1.0):
    """The full m x m inverse of D_{c,C} by the SMW solve of unit vectors."""
    m = L + 3
    return np.column_stack([smw_solve(p, c, L, e, sign) for e in np.eye(m)])


# ---------------------------------------------------- block-Jacobi operator --
class BlockJacobi:
    """M = blockdiag(D_{c,C})^{-1} via dense LU, over all N cells."""

    def __init__(self, diag_blocks):
        self.LU, self.piv = lu_factor(diag_blocks)

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        return lu_solve(self.LU, self.piv, r)

    def apply_T(self, r):
        return lu_solve_T(self.LU, self.piv, r)
