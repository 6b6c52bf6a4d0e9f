"""Matrix-vector products with the assembled dense-block Jacobian.

This is the "standard representation" of section 3 ("Jacobian Complexity")
and section 5.2: every stored block is a dense m x m matrix and y = J x is a
sum of block products over each block row.  Its cost is the N_A formula of
section 3, quadratic in m.

Vectors have shape [nrhs][N][m] (or [N][m] for a single right-hand side).
"""
import numpy as np

from . import assemble, mesh


def _as3(x):
    x = np.asarray(x, dtype=np.float64)
    return x[None] if x.ndim == 2 else x


def bsr_matvec(indptr, indices, data, rows, x, N):
    """y[rows] = sum over the row's blocks of data[b] @ x[indices[b]].

    Returns y of shape [nrhs][len(rows)][m] (block rows in `rows` order).
    """
    x3 = _as3(x)
    nrhs, m = x3.shape[0], x3.shape[2]
    y = np.zeros((nrhs, len(rows), m))
    for r in range(len(rows)):
        for b in range(indptr[r], indptr[r + 1]):
            y[:, r, :] += x3[:, indices[b], :] @ data[b].T
    return y


def matvec(p, nx, ny, L, x, chunk=4096):
    """y = J x over the whole mesh, assembling block rows chunk by chunk."""
    x3 = _as3(x)
    N = nx * ny
    y = np.zeros_like(x3)
    for c0 in range(0, N, chunk):
        cells = range(c0, min(N, c0 + chunk))
        indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L, cells)
        y[:, c0:c0 + len(rows), :] = bsr_matvec(indptr, indices, data, rows, x3, N)
    return y if np.ndim(x) == 3 else y[0]


def matvec_rows(p, nx, ny, L, x, cells):
    """(J x) restricted to the block rows `cells`: [nrhs][len(cells)][m]."""
    indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L, cells)
    return bsr_matvec(indptr, indices, data, rows, x, nx * ny)


def matvec_T(p, nx, ny, L, x, chunk=4096):
    """y = J^T x by scattering D_{c,d}^T x_c into the column block of (c, d).

    A different algorithm from a gather: every block row c adds the product of
    each of its transposed blocks with x_c into the block of y it multiplies.
    """
    x3 = _as3(x)
    N = nx * ny
    y = np.zeros_like(x3)
    for c0 in range(0, N, chunk):
        cells = range(c0, min(N, c0 + chunk))
        indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L, cells)
        for r, c in enumerate(rows):
            for b in range(indptr[r], indptr[r + 1]):
                y[:, indices[b], :] += x3[:, c, :] @ data[b]
    return y if np.ndim(x) == 3 else y[0]


def matvec_T_rows(p, nx, ny, L, x, cells):
    """(J^T x) restricted to the block rows `cells`: [nrhs][len(cells)][m].

    Block column j of J holds the blocks (c, d) whose column cell is j, i.e.
    the diagonal block of j and one block of each neighbour of j; row j of
    J^T is the sum of their transposes applied to x_c.
    """
    x3 = _as3(x)
    out = np.zeros((x3.shape[0], len(cells), L + 3))
    for t, j in enumerate(cells):
        rows = sorted({j} | {nb for nb in mesh.neighbour_table_row(nx, ny, j) if nb >= 0})
        indptr, indices, data, rws = assemble.assemble_bsr(p, nx, ny, L, rows)
        for r, c in enumerate(rws):
            for b in range(indptr[r], indptr[r + 1]):
                if indices[b] == j:
                    out[:, t, :] += x3[:, c, :] @ data[b]
    return out


def dense_matrix(p, nx, ny, L):
    """The full n x n Jacobian (tiny meshes only)."""
    N, m = nx * ny, L + 3
    J = np.zeros((N * m, N * m))
    indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L)
    for r, c in enumerate(rows):
        for b in range(indptr[r], indptr[r + 1]):
            col = indices[b]
            J[c * m:(c + 1) * m, col * m:(col + 1) * m] = data[b]
    return J
