"""The block r1-sparse Jacobian on a general 2-D mesh (test infrastructure).

The block structure comes from the index arrays of the BR1-BSR format
(section 5.1): block_indptr / block_indices list the block columns of every
block row, the diagonal block included.  Every block is sparse plus rank-one
pairs (section 4, "Overall Structure"): the diagonal block as on the
structured mesh, an off-diagonal block a diagonal matrix plus r_off pairs.

This module assembles the dense blocks from those arrays and forms products
and gradients from them (the standard representation of section 3); the
structured product of section 5.2 on the same arrays is in `formats`.
"""
import numpy as np

from . import assemble, mesh


def off_blocks(p):
    """(row, column) of every off-diagonal block, in input order."""
    indptr, indices = p["graph_indptr"], p["graph_indices"]
    rows, cols = [], []
    for c in range(len(indptr) - 1):
        for b in range(indptr[c], indptr[c + 1]):
            if indices[b] != c:
                rows.append(c)
                cols.append(int(indices[b]))
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)


def diag_block(p, c, L):
    """D_cc = S_cc + sum_p u_p v_p^T over the diagonal block's pairs."""
    D = assemble.diagonal_sparse_block(p, c, L)
    for q in range(p["u_diag"].shape[1]):
        D = D + np.outer(p["u_diag"][c, q], p["v_diag"][c, q])
    return D


def off_block(p, o):
    """D = diag(s_nbr[o]) + sum_p u_p v_p^T for off-diagonal block o."""
    D = np.diag(p["s_nbr"][o])
    for q in range(p["u_off"].shape[1]):
        D = D + np.outer(p["u_off"][o, q], p["v_off"][o, q])
    return D


def blocks(p, L):
    """All blocks as (row, column, dense block), in input order."""
    indptr, indices = p["graph_indptr"], p["graph_indices"]
    out, o = [], 0
    for c in range(len(indptr) - 1):
        for b in range(indptr[c], indptr[c + 1]):
            j = int(indices[b])
            if j == c:
                out.append((c, j, diag_block(p, c, L)))
            else:
                out.append((c, j, off_block(p, o)))
                o += 1
    return out


def _as3(x):
    x = np.asarray(x, dtype=np.float64)
    return x[None] if x.ndim == 2 else x


def matvec(p, L, x):
    """y_c = sum over the row's blocks of D x_col."""
    x3 = _as3(x)
    y = np.zeros_like(x3)
    for c, j, D in blocks(p, L):
        y[:, c, :] += x3[:, j, :] @ D.T
    return y if np.ndim(x) == 3 else y[0]


def matvec_T(p, L, x):
    """J^T x by scattering every block's transpose: y_col += D^T x_row."""
    x3 = _as3(x)
    y = np.zeros_like(x3)
    for c, j, D in blocks(p, L):
        y[:, j, :] += x3[:, c, :] @ D
    return y if np.ndim(x) == 3 else y[0]


def dense_matrix(p, L):
    N, m = len(p["graph_indptr"]) - 1, L + 3
    J = np.zeros((N * m, N * m))
    for c, j, D in blocks(p, L):
        J[c * m:(c + 1) * m, j * m:(j + 1) * m] += D
    return J


def diagonal_blocks(p, L, cells=None):
    N = len(p["graph_indptr"]) - 1
    cells = range(N) if cells is None else cells
    return np.array([diag_block(p, c, L) for c in cells])


def smw_view(p):
    """The cell-wise view the Woodbury oracle reads: the diagonal block's
    pairs as the only pairs of a cell (r_off = 0)."""
    q = dict(p)
    q["u"], q["v"] = p["u_diag"], p["v_diag"]
    q["ranks"] = np.array([p["u_diag"].shape[1], 0])
    return q


def grads(p, L, lam, x):
    """Gradients of sum_r w_r . x_r (lambda = J^{-T} w) w.r.t. every array,
    through the dense blocks: G = -sum_r lambda_r[c] x_r[col]^T."""
    lam, x = _as3(lam), _as3(x)
    band, arrow = mesh.pattern(p)
    keys = ["s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u_diag", "v_diag", "u_off", "v_off"]
    if (band, arrow) != (1, 0):
        keys += ["s_band", "s_lev_flow", "s_flow_lev"]
    g = {k: np.zeros_like(p[k]) for k in keys}
    indptr, indices = p["graph_indptr"], p["graph_indices"]
    o = 0
    for c in range(len(indptr) - 1):
        for b in range(indptr[c], indptr[c + 1]):
            j = int(indices[b])
            G = -np.einsum("ri,rj->ij", lam[:, c, :], x[:, j, :])
            if j == c:
                for q in range(p["u_diag"].shape[1]):
                    g["u_diag"][c, q] = G @ p["v_diag"][c, q]
                    g["v_diag"][c, q] = G.T @ p["u_diag"][c, q]
                g["s_diag"][c] = np.diag(G)
                for k in range(L - 1):
                    g["s_sub"][c, k] = G[k + 1, k]
                    g["s_sup"][c, k] = G[k, k + 1]
                for t, (a, bb) in enumerate(assemble.FLOW_PAIRS):
                    g["s_flow"][c, t] = G[L + a, L + bb]
                for jj in range(2, band + 1):
                    for k in range(jj, L):
                        g["s_band"][c, jj - 2, k] = G[k, k - jj]
                    for k in range(0, L - jj):
                        g["s_band"][c, band - 1 + jj - 2, k] = G[k, k + jj]
                if arrow:
                    for i in range(3):
                        g["s_lev_flow"][c, i] = G[:L, L + i]
                        g["s_flow_lev"][c, i] = G[L + i, :L]
                if arrow == 2:
                    g["s_lev_flow"][c, 3, :L - 1] = G[:L - 1, L - 1]
                    g["s_flow_lev"][c, 3, :L - 1] = G[L - 1, :L - 1]
            else:
                for q in range(p["u_off"].shape[1]):
                    g["u_off"][o, q] = G @ p["v_off"][o, q]
                    g["v_off"][o, q] = G.T @ p["u_off"][o, q]
                g["s_nbr"][o] = np.diag(G)
                o += 1
    return g


def structured_values(p, L):
    """Stored values: per cell the diagonal block's pattern and pairs, per
    off-diagonal block its diagonal and pairs."""
    N = len(p["graph_indptr"]) - 1
    n_off = len(p["graph_indices"]) - N
    m = L + 3
    band, arrow = mesh.pattern(p)
    diag_block_vals = m + sum(2 * max(L - j, 0) for j in range(1, band + 1)) + 6 + (6 * L if arrow else 0) + (2 * max(L - 1 - band, 0) if arrow == 2 else 0)
    rd, ro = p["u_diag"].shape[1], p["u_off"].shape[1]
    return N * diag_block_vals + n_off * m + 2 * m * (N * rd + n_off * ro)


def _row_blocks(p, c, L):
    """(column, dense block) of block row c."""
    indptr, indices = p["graph_indptr"], p["graph_indices"]
    o = int(indptr[c]) - c  # off-diagonal blocks of the rows before c
    out = []
    for b in range(indptr[c], indptr[c + 1]):
        j = int(indices[b])
        if j == c:
            out.append((j, diag_block(p, c, L)))
        else:
            out.append((j, off_block(p, o)))
            o += 1
    return out


def matvec_rows(p, L, x, cells):
    """(J x) restricted to the block rows `cells`: [nrhs][len(cells)][m]."""
    x3 = _as3(x)
    out = np.zeros((x3.shape[0], len(cells), L + 3))
    for t, c in enumerate(cells):
        for j, D in _row_blocks(p, c, L):
            out[:, t, :] += x3[:, j, :] @ D.T
    return out


def matvec_T_rows(p, L, x, cells):
    """(J^T x) restricted to the block rows `cells`: row j of J^T sums the
    transposed blocks (c, j) over the cells c whose row lists j (the
    structure is symmetric, so those are j's own neighbours and j)."""
    x3 = _as3(x)
    indptr, indices = p["graph_indptr"], p["graph_indices"]
    out = np.zeros((x3.shape[0], len(cells), L + 3))
    for t, j in enumerate(cells):
        for c in indices[indptr[j]:indptr[j + 1]]:
            for jj, D in _row_blocks(p, int(c), L):
                if jj == j:
                    out[:, t, :] += x3[:, int(c), :] @ D
    return out


def abs_problem(p):
    """The same structure with every value replaced by its absolute value
    (|J| for the componentwise error scale)."""
    return {k: (np.abs(v) if v.dtype.kind == "f" else v) for k, v in p.items()}
