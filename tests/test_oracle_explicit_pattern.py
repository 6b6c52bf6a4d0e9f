"""Pins of the oracle with a general pattern of the diagonal block, shared by
every cell (section 4, "Temporal Source Jacobian": the sparsity of S_cc
follows from the kinetic processes kept; the structured layouts are special
cases).  The pattern is a CSR list of (row, column) entries, values s_cc
[N][nnz] in entry order."""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import rel
from oracle import assemble, blockjacobi, formats, gmres, grads, mesh, ops, storage
from paper_2403_09198_amd import gen

LAYOUTS = [(1, 0), (3, 0), (1, 1), (4, 1), (1, 2), (3, 2)]


def _random(L, seed, **kw):
    return gen.random_pattern(L + 3, seed=seed, **kw)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_explicit_block_matches_a_library_csr(seed):
    L = 9
    ip, ix = _random(L, seed, per_row=3, dense_rows=(L + 1,), dense_cols=(2,))
    p = gen.make_pattern_problem(3, 2, L, ip, ix, seed=seed)
    for c in range(6):
        ref = sp.csr_matrix((p["s_cc"][c], ix, ip), shape=(L + 3, L + 3)).toarray()
        assert np.array_equal(assemble.diagonal_sparse_block(p, c, L), ref)


def test_random_pattern_is_well_formed():
    m = 20
    ip, ix = gen.random_pattern(m, per_row=4, dense_rows=(3,), dense_cols=(7, 11), seed=5)
    assert ip[0] == 0 and len(ip) == m + 1
    for i in range(m):
        cols = list(ix[ip[i]:ip[i + 1]])
        assert len(cols) == len(set(cols)) and i in cols
        assert 7 in cols and 11 in cols
        assert len(cols) >= 4
    assert sorted(ix[ip[3]:ip[4]]) == list(range(m))


@pytest.mark.parametrize("band,arrow", LAYOUTS)
def test_layout_pattern_reproduces_structured_blocks(band, arrow):
    # the structured layouts as explicit patterns: same blocks, and every
    # entry a structured layout can hold lies in the pattern
    L = 8
    q = gen.make_problem(2, 2, L, seed=4, band=band, arrow=arrow)
    ip, ix = gen.layout_pattern(L, band, arrow)
    row = np.repeat(np.arange(L + 3), np.diff(ip))
    for c in range(4):
        A = assemble.diagonal_sparse_block(q, c, L)
        inside = np.zeros_like(A, dtype=bool)
        inside[row, ix] = True
        assert not np.any(A[~inside])
        p = {"pat_indptr": ip, "pat_indices": ix, "s_cc": A[row, ix][None, :].repeat(4, 0)}
        assert np.array_equal(assemble.diagonal_sparse_block(p, c, L), A)


def test_layout_pattern_counts():
    L = 10
    for band, arrow in LAYOUTS:
        ip, _ = gen.layout_pattern(L, band, arrow)
        m = L + 3
        # the structured storage count holds these entries in the diagonal block
        expect = storage.structured_values(1, 1, m, 1, 0, band, arrow) - 2 * m
        assert ip[-1] == expect, (band, arrow)


@pytest.mark.parametrize("seed", [0, 3])
def test_explicit_products_equal_dense(seed):
    nx, ny, L = 4, 3, 7
    ip, ix = _random(L, seed, per_row=2, dense_rows=(0,), dense_cols=(L + 2,))
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=seed, r_diag=2, r_off=1)
    x = gen.make_vector(nx, ny, L, seed=seed)[0]
    J = ops.dense_matrix(p, nx, ny, L)
    assert rel(formats.structured_matvec(p, nx, ny, L, x), J @ x.ravel()) <= 1e-13
    assert rel(ops.matvec(p, nx, ny, L, x).ravel(), J @ x.ravel()) <= 1e-13
    assert rel(ops.matvec_T(p, nx, ny, L, x).ravel(), J.T @ x.ravel()) <= 1e-13


@pytest.mark.parametrize("r_diag", [1, 4])
def test_explicit_woodbury_inverse_times_block_is_identity(r_diag):
    nx, ny, L = 3, 2, 12
    ip, ix = _random(L, 7, per_row=3, dense_rows=(5,), dense_cols=(L,))
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=7, r_diag=r_diag, r_off=1)
    for c in range(nx * ny):
        D = assemble.dense_block(p, c, mesh.C, L)
        assert np.abs(blockjacobi.smw_inverse(p, c, L) @ D - np.eye(L + 3)).max() <= 1e-12


def test_generated_explicit_values_are_dominant():
    nx, ny, L = 6, 6, 60
    ip, ix = _random(L, 2, per_row=6, dense_rows=(L, L + 1), dense_cols=(L - 1,))
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=2)
    for c in range(0, 36, 5):
        A = assemble.diagonal_sparse_block(p, c, L)
        off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
        nbr = np.abs(p["s_nbr"][c]).sum(axis=0)
        assert np.all(np.abs(np.diag(A)) > off + nbr)


def test_gmres_with_explicit_pattern_matches_dense_solve():
    nx, ny, L = 5, 4, 9
    ip, ix = _random(L, 8, per_row=3, dense_rows=(L + 1,), dense_cols=(1,))
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=8, r_diag=3, r_off=2)
    b = gen.make_rhs(nx, ny, L, seed=8)[0]
    M = blockjacobi.BlockJacobi(assemble.diagonal_blocks(p, nx, ny, L))
    res = gmres.gmres(lambda v: ops.matvec(p, nx, ny, L, v), M.apply, b, restart=30, rtol=1e-12)
    J = ops.dense_matrix(p, nx, ny, L)
    assert res.converged
    assert rel(res.x.ravel(), np.linalg.solve(J, b.ravel())) <= 2 * np.linalg.cond(J) * 1e-12


def test_explicit_storage_counts():
    nx, ny, L = 5, 4, 8
    m = L + 3
    ip, ix = _random(L, 1, per_row=2, dense_rows=(3,))
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=1, r_diag=3, r_off=1)
    csr = formats.structured_csr(p, nx, ny, L)
    br1 = formats.structured_br1(p, nx, ny)
    counted = csr[0].size + br1["column_data"].size + br1["row_data"].size
    assert storage.explicit_pattern_values(nx, ny, m, int(ip[-1]), 3, 1) == counted


def test_explicit_gradients_match_finite_differences():
    nx, ny, L, nrhs = 3, 2, 5, 2
    ip, ix = _random(L, 4, per_row=2, dense_rows=(L,), dense_cols=(0,))
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=4, r_diag=2, r_off=1)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=4)
    w = gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=4)
    n = nx * ny * (L + 3)

    def loss_of(q):
        J = ops.dense_matrix(q, nx, ny, L)
        return grads.loss(np.linalg.solve(J, b.reshape(nrhs, n).T).T, w.reshape(nrhs, n))

    J = ops.dense_matrix(p, nx, ny, L)
    x = np.linalg.solve(J, b.reshape(nrhs, n).T).T.reshape(b.shape)
    lam = np.linalg.solve(J.T, w.reshape(nrhs, n).T).T.reshape(b.shape)
    g = grads.structured_grads(p, nx, ny, L, lam, x)
    assert set(g) == set(gen.PATTERN_PROBLEM_FIELDS)
    rng = np.random.default_rng(3)
    h = 1e-6
    for key in gen.PATTERN_PROBLEM_FIELDS:
        for _ in range(8):
            idx = tuple(int(rng.integers(s)) for s in p[key].shape)
            qp = {kk: (vv.copy() if isinstance(vv, np.ndarray) else vv) for kk, vv in p.items()}
            qm = {kk: (vv.copy() if isinstance(vv, np.ndarray) else vv) for kk, vv in p.items()}
            qp[key][idx] += h
            qm[key][idx] -= h
            fd = (loss_of(qp) - loss_of(qm)) / (2 * h)
            assert abs(fd - g[key][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, idx)
