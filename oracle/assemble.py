"""Dense-block assembly of the Jacobian J = S + sum_blocks u v^T.

Section 4 ("Overall Structure"): every non-zero m x m block of J is an
r1-sparse matrix, the sum of a sparse block and rank-one updates (the
definition of r1-sparsity in section 4.1):

    D_{c,d} = S_{c,d} + sum over the block's pairs p of  u_p v_p^T.

S_{c,C} (the diagonal block) has a full diagonal, a band coupling levels k, k'
with 0 < |k - k'| <= band (band = 1: tridiagonal; section 4, "Temporal Source
Jacobian": level-changing processes up to a threshold jump give a banded
pattern), a dense 3 x 3 corner for the flow unknowns L, L+1, L+2 and, with
the arrow option, dense coupling between the level rows and the flow columns
and between the flow rows and the level columns.  With arrow = 2 the last
level a = L - 1 is the atom density (the DRa processes of the same passage:
each molecule level's row depends on its own density, the atom density and
the temperature, and the atom's row on every level): a dense atom column
S[k][a] and atom row S[a][k] over the molecule levels k < a are added to the
block (the generator draws the band entries that reach the atom as zero, so
every entry has one source; the block is the sum of its parts).  A general
pattern shared by every cell (explicit CSR pattern, values s_cc in entry
order) replaces all of these.  S_{c,d} for d != C is diagonal.

The result is stored in the paper's BSR format (section 5.1): block_indptr,
block_indices (ascending block columns within a block row) and a 3-D data
array [n_blocks][m][m].
"""
import numpy as np

from . import mesh

FLOW_PAIRS = ((0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1))


def diagonal_sparse_block(p, c: int, L: int) -> np.ndarray:
    """S_{c,C} as a dense m x m array (sparse pattern, zeros elsewhere)."""
    m = L + 3
    ep = mesh.explicit_pattern(p)
    if ep is not None:  # a general pattern: entry e of row i sits at column indices[e]
        indptr, indices = ep
        A = np.zeros((m, m))
        for i in range(m):
            for e in range(indptr[i], indptr[i + 1]):
                A[i, indices[e]] = p["s_cc"][c, e]
        return A
    A = np.zeros((m, m))
    A[np.arange(m), np.arange(m)] = p["s_diag"][c]
    for k in range(L - 1):
        A[k + 1, k] = p["s_sub"][c, k]
        A[k, k + 1] = p["s_sup"][c, k]
    for t, (i, j) in enumerate(FLOW_PAIRS):
        A[L + i, L + j] = p["s_flow"][c, t]
    band, arrow = mesh.pattern(p)
    for j in range(2, band + 1):
        for k in range(j, L):
            A[k, k - j] = p["s_band"][c, j - 2, k]
        for k in range(0, L - j):
            A[k, k + j] = p["s_band"][c, band - 1 + j - 2, k]
    if arrow:
        for i in range(3):
            A[:L, L + i] = p["s_lev_flow"][c, i]
            A[L + i, :L] = p["s_flow_lev"][c, i]
    if arrow == 2:
        a = L - 1
        A[:a, a] += p["s_lev_flow"][c, 3, :a]
        A[a, :a] += p["s_flow_lev"][c, 3, :a]
    return A


def sparse_block(p, c: int, d: int, L: int) -> np.ndarray:
    """S_{c,d} as a dense m x m array."""
    if d == mesh.C:
        return diagonal_sparse_block(p, c, L)
    return np.diag(p["s_nbr"][c, mesh.NBR_SLOT[d]])


def dense_block(p, c: int, d: int, L: int) -> np.ndarray:
    """D_{c,d} = S_{c,d} + sum_p u_p v_p^T over the pairs of block (c, d)."""
    D = sparse_block(p, c, d, L)
    a, cnt = mesh.pair_range(p, d)
    for q in range(a, a + cnt):
        D = D + np.outer(p["u"][c, q], p["v"][c, q])
    return D


def assemble_bsr(p, nx: int, ny: int, L: int, cells=None):
    """Assemble the block rows of `cells` (default: all) in BSR format.

    Returns (block_indptr, block_indices, data, rows): `rows` are the block-row
    cell numbers in order, block_indptr indexes into block_indices/data
    relative to that list of rows.
    """
    if cells is None:
        cells = range(nx * ny)
    cells = list(cells)
    indptr = [0]
    indices = []
    blocks = []
    for c in cells:
        for d in (mesh.S, mesh.W, mesh.C, mesh.E, mesh.N):
            nb = mesh.neighbour(nx, ny, c, d)
            if nb < 0:
                continue
            indices.append(nb)
            blocks.append(dense_block(p, c, d, L))
        indptr.append(len(indices))
    m = L + 3
    data = np.array(blocks).reshape(len(blocks), m, m)
    return (np.array(indptr, dtype=np.int64), np.array(indices, dtype=np.int64),
            data, np.array(cells, dtype=np.int64))


def diagonal_blocks(p, nx: int, ny: int, L: int, cells=None) -> np.ndarray:
    """[len(cells)][m][m] diagonal blocks D_{c,C} (the block-Jacobi blocks)."""
    if cells is None:
        cells = range(nx * ny)
    return np.array([dense_block(p, c, mesh.C, L) for c in cells])
