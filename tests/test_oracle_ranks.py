"""Pins of the oracle with several rank-one pairs per block (section 4,
"Overall Structure": nine on a diagonal block, two on an off-diagonal one)."""
import numpy as np
import pytest

from conftest import rel
from oracle import assemble, blockjacobi, formats, gmres, grads, mesh, ops, storage
from paper_2403_09198_amd import gen

RANKS = [(9, 2), (3, 1), (2, 0)]


@pytest.mark.parametrize("r_diag,r_off", RANKS)
def test_structured_product_equals_assembled(r_diag, r_off):
    nx, ny, L = 4, 3, 6
    p = gen.make_problem(nx, ny, L, seed=21, r_diag=r_diag, r_off=r_off)
    x = gen.make_vector(nx, ny, L, seed=2)[0]
    J = ops.dense_matrix(p, nx, ny, L)
    assert rel(formats.structured_matvec(p, nx, ny, L, x), J @ x.ravel()) <= 1e-13
    assert rel(ops.matvec(p, nx, ny, L, x).ravel(), J @ x.ravel()) <= 1e-13
    assert rel(ops.matvec_T(p, nx, ny, L, x).ravel(), J.T @ x.ravel()) <= 1e-13


def test_paper_pair_counts_in_br1_bsr():
    # a diagonal block carries 9 pairs, an off-diagonal block 2: the
    # pair_indptr differences of the BR1-BSR structure
    nx, ny, L = 3, 3, 4
    p = gen.make_problem(nx, ny, L, seed=1, r_diag=9, r_off=2)
    br1 = formats.structured_br1(p, nx, ny)
    counts = np.diff(br1["pair_indptr"])
    cols = br1["block_indices"]
    rows = np.repeat(np.arange(nx * ny), np.diff(br1["block_indptr"]))
    assert np.all(counts[cols == rows] == 9) and np.all(counts[cols != rows] == 2)
    # the centre cell has four neighbours: 9 + 4 * 2 pairs in its block row
    assert br1["column_pair_indptr"][5] - br1["column_pair_indptr"][4] == 17


def test_rank_one_sum_is_rank_r():
    p = gen.make_problem(2, 2, 10, seed=3, r_diag=9, r_off=2)
    D = assemble.dense_block(p, 1, mesh.C, 10) - assemble.sparse_block(p, 1, mesh.C, 10)
    assert np.linalg.matrix_rank(D, tol=1e-10) == 9
    O = assemble.dense_block(p, 1, mesh.W, 10) - assemble.sparse_block(p, 1, mesh.W, 10)
    assert np.linalg.matrix_rank(O, tol=1e-10) == 2


@pytest.mark.parametrize("r_diag", [9, 3])
def test_woodbury_inverse_times_block_is_identity(r_diag):
    nx, ny, L = 3, 2, 20
    p = gen.make_problem(nx, ny, L, seed=5, r_diag=r_diag, r_off=2)
    for c in range(nx * ny):
        D = assemble.dense_block(p, c, mesh.C, L)
        assert np.abs(blockjacobi.smw_inverse(p, c, L) @ D - np.eye(L + 3)).max() <= 1e-12
    Mplus = blockjacobi.smw_inverse(p, 0, L, sign=+1.0)
    assert np.abs(Mplus @ assemble.dense_block(p, 0, mesh.C, L) - np.eye(L + 3)).max() > 1e-6


def test_gmres_with_paper_ranks_matches_dense_solve():
    nx, ny, L = 8, 6, 9
    p = gen.make_problem(nx, ny, L, seed=7, r_diag=9, r_off=2)
    b = gen.make_rhs(nx, ny, L, seed=7)[0]
    D = assemble.diagonal_blocks(p, nx, ny, L)
    M = blockjacobi.BlockJacobi(D)
    res = gmres.gmres(lambda v: ops.matvec(p, nx, ny, L, v), M.apply, b, restart=30, rtol=1e-12)
    J = ops.dense_matrix(p, nx, ny, L)
    assert res.converged
    assert rel(res.x.ravel(), np.linalg.solve(J, b.ravel())) <= 2 * np.linalg.cond(J) * 1e-12


def test_storage_counts_with_ranks():
    nx, ny, L = 5, 4, 6
    m = L + 3
    for r_diag, r_off in RANKS:
        p = gen.make_problem(nx, ny, L, seed=1, r_diag=r_diag, r_off=r_off)
        csr = formats.structured_csr(p, nx, ny, L)
        br1 = formats.structured_br1(p, nx, ny)
        counted = csr[0].size + br1["column_data"].size + br1["row_data"].size
        assert storage.structured_values(nx, ny, m, r_diag, r_off) == counted
        s = [storage.structured_values(nx, ny, mm, r_diag, r_off) for mm in (m - 1, m, m + 1)]
        assert s[2] - 2 * s[1] + s[0] == 0


def test_gradients_with_ranks_match_finite_differences():
    nx, ny, L, nrhs = 3, 2, 3, 2
    p = gen.make_problem(nx, ny, L, seed=9, r_diag=3, r_off=2)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=9)
    w = gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=9)
    n = nx * ny * (L + 3)

    def loss_of(q):
        J = ops.dense_matrix(q, nx, ny, L)
        return grads.loss(np.linalg.solve(J, b.reshape(nrhs, n).T).T, w.reshape(nrhs, n))

    J = ops.dense_matrix(p, nx, ny, L)
    x = np.linalg.solve(J, b.reshape(nrhs, n).T).T.reshape(b.shape)
    lam = np.linalg.solve(J.T, w.reshape(nrhs, n).T).T.reshape(b.shape)
    g = grads.structured_grads(p, nx, ny, L, lam, x)
    ex = gen.block_exists(nx, ny)
    slots = gen.pair_slots(3, 2)
    rng = np.random.default_rng(1)
    h = 1e-6
    for key in ("u", "v"):
        for _ in range(8):
            c = int(rng.integers(nx * ny))
            d = int(rng.choice(np.flatnonzero(ex[c])))
            a, cnt = slots[d]
            q = a + int(rng.integers(cnt))
            k = int(rng.integers(L + 3))
            qp = {kk: vv.copy() for kk, vv in p.items()}
            qm = {kk: vv.copy() for kk, vv in p.items()}
            qp[key][c, q, k] += h
            qm[key][c, q, k] -= h
            fd = (loss_of(qp) - loss_of(qm)) / (2 * h)
            assert abs(fd - g[key][c, q, k]) <= 1e-6 * max(1.0, abs(fd))
