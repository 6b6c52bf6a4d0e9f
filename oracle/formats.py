"""Storage formats of section 5.1 and the structured matvec of section 5.2.

* CSR: data / indices / indptr of the non-zeros in row-major order.
* r1-sparse matrix: CSR data plus r1_columns / r1_rows, one row per rank-one
  update (the column vectors u and the row vectors v of A + sum u v^T).
* BSR: block_indices / block_indptr and a 3-D data array of non-zero blocks.
* BR1-BSR: block_indices / block_indptr of the blocks that carry rank-one
  pairs, column_data (u) and row_data (v) for every pair, pair_indptr (pairs
  of each block) and the auxiliary column_pair_indptr (pairs of each block
  row).

The structured product of section 5.2 adds the CSR product of the fully
sparse part to the block rank-one product: for every pair first the scalar
coefficient v . x_{block column}, then the accumulation coefficient * u into
the block row.
"""
import numpy as np

from . import assemble, mesh


# ---------------------------------------------------------------- CSR / BSR --
def dense_to_csr(A):
    """CSR arrays of the non-zeros of a dense matrix, row by row."""
    A = np.asarray(A)
    data, indices, indptr = [], [], [0]
    for i in range(A.shape[0]):
        for j in range(A.shape[1]):
            if A[i, j] != 0:
                data.append(A[i, j])
                indices.append(j)
        indptr.append(len(data))
    return np.array(data), np.array(indices, dtype=np.int64), np.array(indptr, dtype=np.int64)


def csr_matvec(data, indices, indptr, x):
    """Row-wise dot products of a CSR matrix with x (section 5.2, CSR part)."""
    x = np.asarray(x, dtype=np.float64)
    nrows = len(indptr) - 1
    y = np.zeros(nrows)
    for i in range(nrows):
        acc = 0.0
        for t in range(indptr[i], indptr[i + 1]):
            acc += data[t] * x[indices[t]]
        y[i] = acc
    return y


def csr_to_dense(data, indices, indptr, ncols):
    nrows = len(indptr) - 1
    A = np.zeros((nrows, ncols))
    for i in range(nrows):
        for t in range(indptr[i], indptr[i + 1]):
            A[i, indices[t]] = data[t]
    return A


def r1_sparse(U, V):
    """r1_columns / r1_rows of the update sum_k U[:,k] V[:,k]^T: one row per
    rank-one term, holding that term's column vector / row vector."""
    return np.array(np.asarray(U).T), np.array(np.asarray(V).T)


def r1_sparse_matvec(csr, r1_columns, r1_rows, x):
    """(A + sum_k u_k v_k^T) x with A in CSR form."""
    y = csr_matvec(*csr, x)
    for u, v in zip(r1_columns, r1_rows):
        y = y + u * float(np.dot(v, x))
    return y


def dense_to_bsr(A, bs):
    """BSR arrays (block_indices, block_indptr, data) of the non-zero bs x bs
    blocks of A, block row by block row."""
    A = np.asarray(A)
    nbr, nbc = A.shape[0] // bs, A.shape[1] // bs
    indices, indptr, data = [], [0], []
    for I in range(nbr):
        for J in range(nbc):
            blk = A[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
            if np.any(blk != 0):
                indices.append(J)
                data.append(blk.copy())
        indptr.append(len(indices))
    return (np.array(indices, dtype=np.int64), np.array(indptr, dtype=np.int64),
            np.array(data))


# -------------------------------------------------------------- BR1-BSR ------
def br1_bsr(block_pairs, nblock_rows):
    """BR1-BSR arrays from a list of (block_row, block_col, [(u, v), ...]).

    Blocks must be listed block row by block row.  Returns a dict with
    block_indices, block_indptr, column_data, row_data, pair_indptr and
    column_pair_indptr.
    """
    block_indices, column_data, row_data = [], [], []
    block_indptr = np.zeros(nblock_rows + 1, dtype=np.int64)
    pair_indptr = [0]
    pairs_per_row = np.zeros(nblock_rows, dtype=np.int64)
    last_row = -1
    for (I, J, pairs) in block_pairs:
        if I < last_row:
            raise ValueError("blocks must be ordered by block row")
        last_row = I
        block_indices.append(J)
        block_indptr[I + 1] += 1
        for (u, v) in pairs:
            column_data.append(np.asarray(u, dtype=np.float64))
            row_data.append(np.asarray(v, dtype=np.float64))
        pair_indptr.append(pair_indptr[-1] + len(pairs))
        pairs_per_row[I] += len(pairs)
    return {
        "block_indices": np.array(block_indices, dtype=np.int64),
        "block_indptr": np.cumsum(block_indptr),
        "column_data": np.array(column_data),
        "row_data": np.array(row_data),
        "pair_indptr": np.array(pair_indptr, dtype=np.int64),
        "column_pair_indptr": np.concatenate([[0], np.cumsum(pairs_per_row)]),
    }


def br1_matvec(br1, x, column_size, row_size, y=None):
    """Block rank-one product of section 5.2, accumulated into y.

    For each block row: every pair's coefficient v . x_J (J = the block's
    column), kept in a column_coeffs buffer in pair order; then every pair of
    the row adds coefficient * u to the row's output segment.  As in the
    paper the product is accumulated into an output that may already hold
    the sparse part's product.
    """
    x = np.asarray(x, dtype=np.float64)
    nrows = len(br1["block_indptr"]) - 1
    if y is None:
        y = np.zeros(nrows * column_size)
    coeffs = np.zeros(len(br1["row_data"]))
    for I in range(nrows):
        for b in range(br1["block_indptr"][I], br1["block_indptr"][I + 1]):
            J = br1["block_indices"][b]
            xJ = x[J * row_size:(J + 1) * row_size]
            for q in range(br1["pair_indptr"][b], br1["pair_indptr"][b + 1]):
                coeffs[q] = float(np.dot(br1["row_data"][q], xJ))
        seg = slice(I * column_size, (I + 1) * column_size)
        for q in range(br1["column_pair_indptr"][I], br1["column_pair_indptr"][I + 1]):
            y[seg] += coeffs[q] * br1["column_data"][q]
    return y, coeffs


# ------------------------------------------ structured Jacobian, both parts --
def _add_atom(row, p, c, k, L, base):
    """Level row k of cell c gains the atom's column (k < a) or, for the
    atom a = L - 1 itself, its row over the molecule levels (arrow = 2: the
    DRa couplings of section 4, "Temporal Source Jacobian"), added to what
    the band already put there."""
    a = L - 1
    if k < a:
        row[base + a] = row.get(base + a, 0.0) + p["s_lev_flow"][c, 3, k]
    else:
        for kk in range(a):
            row[base + kk] = row.get(base + kk, 0.0) + p["s_flow_lev"][c, 3, kk]


def structured_csr(p, nx, ny, L):
    """CSR of the fully sparse part S (section 4, Fig. 7(b)), built from the
    per-cell pattern directly (no dense block is formed)."""
    N, m = nx * ny, L + 3
    data, indices, indptr = [], [], [0]
    ep = mesh.explicit_pattern(p)
    for c in range(N):
        for k in range(m):
            row = {}
            if ep is not None:  # a general pattern: row k's entries as listed
                pi, pj = ep
                for e in range(pi[k], pi[k + 1]):
                    row[c * m + int(pj[e])] = p["s_cc"][c, e]
                for d in (mesh.S, mesh.W, mesh.E, mesh.N):
                    nb = mesh.neighbour(nx, ny, c, d)
                    if nb >= 0:
                        row[nb * m + k] = p["s_nbr"][c, mesh.NBR_SLOT[d], k]
                for col in sorted(row):
                    data.append(row[col])
                    indices.append(col)
                indptr.append(len(data))
                continue
            # diagonal block pattern
            row[c * m + k] = p["s_diag"][c, k]
            if k < L:
                if k >= 1:
                    row[c * m + k - 1] = p["s_sub"][c, k - 1]
                if k <= L - 2:
                    row[c * m + k + 1] = p["s_sup"][c, k]
            else:
                i = k - L
                for t, (a, b) in enumerate(assemble.FLOW_PAIRS):
                    if a == i:
                        row[c * m + L + b] = p["s_flow"][c, t]
            band, arrow = mesh.pattern(p)
            if k < L:
                for j in range(2, band + 1):
                    if k - j >= 0:
                        row[c * m + k - j] = p["s_band"][c, j - 2, k]
                    if k + j < L:
                        row[c * m + k + j] = p["s_band"][c, band - 1 + j - 2, k]
                if arrow:
                    for i in range(3):
                        row[c * m + L + i] = p["s_lev_flow"][c, i, k]
                if arrow == 2:
                    _add_atom(row, p, c, k, L, c * m)
            elif arrow:
                for kk in range(L):
                    row[c * m + kk] = p["s_flow_lev"][c, k - L, kk]
            # neighbour blocks are diagonal
            for d in (mesh.S, mesh.W, mesh.E, mesh.N):
                nb = mesh.neighbour(nx, ny, c, d)
                if nb >= 0:
                    row[nb * m + k] = p["s_nbr"][c, mesh.NBR_SLOT[d], k]
            for col in sorted(row):
                data.append(row[col])
                indices.append(col)
            indptr.append(len(data))
    return np.array(data), np.array(indices, dtype=np.int64), np.array(indptr, dtype=np.int64)


def structured_br1(p, nx, ny):
    """BR1-BSR arrays of the block rank-one part (all pairs of every block)."""
    N = nx * ny
    blocks = []
    for c in range(N):
        for d in (mesh.S, mesh.W, mesh.C, mesh.E, mesh.N):
            nb = mesh.neighbour(nx, ny, c, d)
            if nb >= 0:
                a, cnt = mesh.pair_range(p, d)
                blocks.append((c, nb, [(p["u"][c, q], p["v"][c, q]) for q in range(a, a + cnt)]))
    return br1_bsr(blocks, N)


def structured_matvec(p, nx, ny, L, x, csr=None, br1=None):
    """y = S x + sum_blocks u (v . x): CSR product then the BR1 product
    accumulated on top (section 5.2).  x is a flat vector of length N*m."""
    m = L + 3
    if csr is None:
        csr = structured_csr(p, nx, ny, L)
    if br1 is None:
        br1 = structured_br1(p, nx, ny)
    y = csr_matvec(*csr, np.ravel(x))
    y, _ = br1_matvec(br1, np.ravel(x), m, m, y=y)
    return y


# -------------------------------------------------------- general mesh --
def graph_csr(p, L):
    """CSR of the fully sparse part S on a general mesh (per-cell diagonal
    block pattern, diagonal off-diagonal blocks), row by row."""
    indptr, indices = p["graph_indptr"], p["graph_indices"]
    N, m = len(indptr) - 1, L + 3
    band, arrow = mesh.pattern(p)
    data, cols, rowptr = [], [], [0]
    for c in range(N):
        offs = []  # column cells of the row's off-diagonal blocks, in order
        for b in range(indptr[c], indptr[c + 1]):
            j = int(indices[b])
            if j != c:
                offs.append(j)
        # off-block numbers of this row: consecutive, starting after all
        # off blocks of earlier rows
        first = int(indptr[c]) - c
        for k in range(m):
            row = {c * m + k: p["s_diag"][c, k]}
            if k < L:
                if k >= 1:
                    row[c * m + k - 1] = p["s_sub"][c, k - 1]
                if k <= L - 2:
                    row[c * m + k + 1] = p["s_sup"][c, k]
                for j in range(2, band + 1):
                    if k - j >= 0:
                        row[c * m + k - j] = p["s_band"][c, j - 2, k]
                    if k + j < L:
                        row[c * m + k + j] = p["s_band"][c, band - 1 + j - 2, k]
                if arrow:
                    for i in range(3):
                        row[c * m + L + i] = p["s_lev_flow"][c, i, k]
                if arrow == 2:
                    _add_atom(row, p, c, k, L, c * m)
            else:
                i = k - L
                for t, (a, b) in enumerate(assemble.FLOW_PAIRS):
                    if a == i:
                        row[c * m + L + b] = p["s_flow"][c, t]
                if arrow:
                    for kk in range(L):
                        row[c * m + kk] = p["s_flow_lev"][c, i, kk]
            for t, j in enumerate(offs):
                row[j * m + k] = p["s_nbr"][first + t, k]
            for col in sorted(row):
                data.append(row[col])
                cols.append(col)
            rowptr.append(len(data))
    return np.array(data), np.array(cols, dtype=np.int64), np.array(rowptr, dtype=np.int64)


def graph_br1(p):
    """BR1-BSR arrays of the rank-one part on a general mesh."""
    indptr, indices = p["graph_indptr"], p["graph_indices"]
    blocks, o = [], 0
    for c in range(len(indptr) - 1):
        for b in range(indptr[c], indptr[c + 1]):
            j = int(indices[b])
            if j == c:
                pairs = list(zip(p["u_diag"][c], p["v_diag"][c]))
            else:
                pairs = list(zip(p["u_off"][o], p["v_off"][o]))
                o += 1
            blocks.append((c, j, pairs))
    return br1_bsr(blocks, len(indptr) - 1)


def graph_matvec(p, L, x, csr=None, br1=None):
    """y = S x (CSR) + the BR1 product accumulated on top (section 5.2)."""
    m = L + 3
    if csr is None:
        csr = graph_csr(p, L)
    if br1 is None:
        br1 = graph_br1(p)
    y = csr_matvec(*csr, np.ravel(x))
    y, _ = br1_matvec(br1, np.ravel(x), m, m, y=y)
    return y
