"""Pins of the oracle's block-Jacobi (dense LU and SMW forms), GMRES,
gradients and storage counts."""
import numpy as np
import pytest
import scipy.linalg as sla

from conftest import rel
from oracle import assemble, blockjacobi, formats, gmres, grads, ops, storage
from paper_2403_09198_amd import gen


# ---------------------------------------------------------- dense LU --------
def test_lu_solve_matches_lapack():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 9, 9))
    A[:, 0, 0] = 0.0  # forces a row swap at the first step
    b = rng.standard_normal((40, 9))
    LU, piv = blockjacobi.lu_factor(A)
    x = blockjacobi.lu_solve(LU, piv, b)
    xt = blockjacobi.lu_solve_T(LU, piv, b)
    for i in range(40):
        assert rel(x[i], np.linalg.solve(A[i], b[i])) <= 1e-12
        assert rel(xt[i], np.linalg.solve(A[i].T, b[i])) <= 1e-12


def test_lu_factor_reconstructs_block():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((5, 7, 7))
    LU, piv = blockjacobi.lu_factor(A)
    for i in range(5):
        Lm = np.tril(LU[i], -1) + np.eye(7)
        Um = np.triu(LU[i])
        PA = A[i].copy()
        for k in range(7):
            PA[[k, piv[i, k]]] = PA[[piv[i, k], k]]
        assert np.allclose(Lm @ Um, PA, atol=1e-13)


def test_singular_block_raises():
    A = np.zeros((1, 3, 3))
    with pytest.raises(blockjacobi.SingularBlock):
        blockjacobi.lu_factor(A)


# ------------------------------------------------------------- SMW ----------
def test_tridiag_matches_solve_banded():
    rng = np.random.default_rng(2)
    n = 17
    a = 5 + rng.random(n)
    b = rng.standard_normal(n - 1)
    c = rng.standard_normal(n - 1)
    r = rng.standard_normal(n)
    ab = np.zeros((3, n))
    ab[0, 1:] = c
    ab[1] = a
    ab[2, :-1] = b
    assert rel(blockjacobi.tridiag_solve(a, b, c, r), sla.solve_banded((1, 1), ab, r)) <= 1e-14


@pytest.mark.parametrize("nx,ny,L", [(16, 16, 8), (2, 3, 1), (3, 2, 61)])
def test_smw_inverse_times_block_is_identity(nx, ny, L):
    # self-check 2: the SMW inverse of D_cc times D_cc is I to 1e-12
    p = gen.make_problem(nx, ny, L, seed=5)
    m = L + 3
    for c in (0, nx * ny // 2, nx * ny - 1):
        D = assemble.dense_block(p, c, 2, L)
        Minv = blockjacobi.smw_inverse(p, c, L)
        assert np.abs(Minv @ D - np.eye(m)).max() <= 1e-12


def test_printed_smw_sign_does_not_invert():
    # the printed "+" in eq. SMW and in the assembly step does not give an inverse
    p = gen.make_problem(4, 4, 8, seed=5)
    D = assemble.dense_block(p, 5, 2, 8)
    Mplus = blockjacobi.smw_inverse(p, 5, 8, sign=+1.0)
    assert np.abs(Mplus @ D - np.eye(11)).max() > 1e-6


def test_smw_with_zero_update_is_sparse_solve():
    p = gen.make_problem(3, 3, 6, seed=8)
    p["u"][:] = 0.0
    r = np.random.default_rng(0).standard_normal(9)
    S = assemble.sparse_block(p, 4, 2, 6)
    assert rel(blockjacobi.smw_solve(p, 4, 6, r), np.linalg.solve(S, r)) <= 1e-13


def test_block_jacobi_operator():
    nx, ny, L = 4, 3, 5
    p = gen.make_problem(nx, ny, L, seed=3)
    D = assemble.diagonal_blocks(p, nx, ny, L)
    M = blockjacobi.BlockJacobi(D)
    r = gen.make_vector(nx, ny, L, nrhs=2, seed=1)
    z = M.apply(r)
    zt = M.apply_T(r)
    for c in range(nx * ny):
        assert rel(D[c] @ z[0, c], r[0, c]) <= 1e-13
        assert rel(D[c].T @ zt[1, c], r[1, c]) <= 1e-13
        assert rel(z[1, c], blockjacobi.smw_solve(p, c, L, r[1, c])) <= 1e-12


# ------------------------------------------------------------ GMRES ---------
def _operators(p, nx, ny, L, trans=False):
    D = assemble.diagonal_blocks(p, nx, ny, L)
    M = blockjacobi.BlockJacobi(D)
    if trans:
        return (lambda v: ops.matvec_T(p, nx, ny, L, v)), M.apply_T
    return (lambda v: ops.matvec(p, nx, ny, L, v)), M.apply


def test_gmres_matches_dense_solve_small_workload():
    # self-check 3: GMRES(30) to 1e-10 agrees with a brute-force dense solve
    nx, ny, L = 16, 16, 8
    p = gen.make_problem(nx, ny, L, seed=0)
    b = gen.make_rhs(nx, ny, L, seed=0)[0]
    A, M = _operators(p, nx, ny, L)
    res = gmres.gmres(A, M, b, restart=30, rtol=1e-10)
    assert res.converged and res.rel_residual <= 1e-10
    J = ops.dense_matrix(p, nx, ny, L)
    x_star = np.linalg.solve(J, b.ravel())
    kappa = np.linalg.cond(J)
    assert rel(res.x.ravel(), x_star) <= 2 * kappa * 1e-10
    assert res.iters < 30


def test_gmres_single_cell_is_one_iteration():
    # block-Jacobi is the exact inverse on a 1x1 mesh
    p = gen.make_problem(1, 1, 12, seed=1)
    b = gen.make_rhs(1, 1, 12, seed=1)[0]
    A, M = _operators(p, 1, 1, 12)
    res = gmres.gmres(A, M, b, restart=10, rtol=1e-12)
    assert res.converged and res.iters == 1


def test_gmres_decoupled_blocks_is_one_iteration():
    nx, ny, L = 4, 3, 5
    p = gen.make_problem(nx, ny, L, seed=2)
    p["s_nbr"][:] = 0.0
    for d in (0, 1, 3, 4):
        p["u"][:, d] = 0.0
        p["v"][:, d] = 0.0
    b = gen.make_rhs(nx, ny, L, seed=2)[0]
    A, M = _operators(p, nx, ny, L)
    res = gmres.gmres(A, M, b, restart=10, rtol=1e-12)
    assert res.converged and res.iters == 1


def test_gmres_stress_restarts():
    # inv_dt = 1: not diagonally dominant; GMRES(5) needs several cycles
    nx, ny, L = 6, 5, 4
    p = gen.make_problem(nx, ny, L, seed=4, inv_dt=1.0)
    b = gen.make_rhs(nx, ny, L, seed=4)[0]
    A, M = _operators(p, nx, ny, L)
    res = gmres.gmres(A, M, b, restart=5, rtol=1e-10, max_cycles=500)
    assert res.converged and res.cycles > 1
    J = ops.dense_matrix(p, nx, ny, L)
    assert rel(res.x.ravel(), np.linalg.solve(J, b.ravel())) <= 2 * np.linalg.cond(J) * 1e-10


def test_gmres_transposed_system():
    nx, ny, L = 5, 4, 3
    p = gen.make_problem(nx, ny, L, seed=6)
    w = gen.make_loss_weights(nx, ny, L, seed=6)[0]
    A, M = _operators(p, nx, ny, L, trans=True)
    res = gmres.gmres(A, M, w, restart=20, rtol=1e-12)
    J = ops.dense_matrix(p, nx, ny, L)
    assert res.converged
    assert rel(res.x.ravel(), np.linalg.solve(J.T, w.ravel())) <= 1e-10


def test_gmres_noconv_reports_failure():
    p = gen.make_problem(4, 4, 3, seed=1, inv_dt=1.0)
    b = gen.make_rhs(4, 4, 3, seed=1)[0]
    A, M = _operators(p, 4, 4, 3)
    res = gmres.gmres(A, M, b, restart=1, rtol=1e-15, max_cycles=1)
    assert not res.converged and res.rel_residual < 1.0


# --------------------------------------------------------- gradients --------
def test_gradients_match_finite_differences_of_dense_solve():
    nx, ny, L, nrhs = 3, 2, 3, 2
    p = gen.make_problem(nx, ny, L, seed=7)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=7)
    w = gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=7)
    n = nx * ny * (L + 3)

    def loss_of(q, bb):
        J = ops.dense_matrix(q, nx, ny, L)
        X = np.linalg.solve(J, bb.reshape(nrhs, n).T).T
        return grads.loss(X, w.reshape(nrhs, n))

    J = ops.dense_matrix(p, nx, ny, L)
    x = np.linalg.solve(J, b.reshape(nrhs, n).T).T.reshape(b.shape)
    lam = np.linalg.solve(J.T, w.reshape(nrhs, n).T).T.reshape(b.shape)
    g = grads.structured_grads(p, nx, ny, L, lam, x)
    h = 1e-6
    ex = gen.block_exists(nx, ny)
    rng = np.random.default_rng(0)
    for key in ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v"):
        flat = p[key].reshape(-1)
        mask = np.ones(flat.size, dtype=bool)
        if key in ("u", "v"):
            mask = np.repeat(ex.reshape(-1), L + 3)
        if key == "s_nbr":
            mask = np.repeat(ex[:, [0, 1, 3, 4]].reshape(-1), L + 3)
        cand = np.flatnonzero(mask)
        for i in rng.choice(cand, size=min(6, cand.size), replace=False):
            q1 = {k: v.copy() for k, v in p.items()}
            q2 = {k: v.copy() for k, v in p.items()}
            q1[key].reshape(-1)[i] += h
            q2[key].reshape(-1)[i] -= h
            fd = (loss_of(q1, b) - loss_of(q2, b)) / (2 * h)
            assert abs(fd - g[key].reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), key
    # dLoss/db is lambda: check one direction
    db = rng.standard_normal(b.shape)
    fd = (loss_of(p, b + h * db) - loss_of(p, b - h * db)) / (2 * h)
    assert abs(fd - float(np.sum(lam * db))) <= 1e-7 * max(1.0, abs(fd))


# ----------------------------------------------------------- storage --------
@pytest.mark.parametrize("nx,ny", [(16, 16), (256, 128), (1, 1), (3, 1)])
def test_block_count_closed_form(nx, ny):
    assert storage.n_blocks(nx, ny) == 5 * nx * ny - 2 * nx - 2 * ny


def test_storage_counts_match_assembled_structures():
    nx, ny, L = 5, 4, 6
    m = L + 3
    p = gen.make_problem(nx, ny, L, seed=1)
    indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L)
    assert storage.bsr_values(nx, ny, m) == data.size
    csr = formats.structured_csr(p, nx, ny, L)
    br1 = formats.structured_br1(p, nx, ny)
    counted = csr[0].size + br1["column_data"].size + br1["row_data"].size
    assert storage.structured_values(nx, ny, m) == counted


def test_storage_growth_linear_vs_quadratic():
    # self-check 4: second difference in m is 0 (structured) and 2B (BSR)
    nx, ny = 16, 16
    B = storage.n_blocks(nx, ny)
    for m in range(5, 40):
        s = [storage.structured_values(nx, ny, mm) for mm in (m - 1, m, m + 1)]
        q = [storage.bsr_values(nx, ny, mm) for mm in (m - 1, m, m + 1)]
        assert s[2] - 2 * s[1] + s[0] == 0
        assert q[2] - 2 * q[1] + q[0] == 2 * B
