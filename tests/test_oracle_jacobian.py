"""Pins of the oracle's Jacobian assembly and matvecs."""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import golden_problem, rel
from oracle import assemble, formats, mesh, ops
from paper_2403_09198_amd import gen


@pytest.mark.parametrize("name", ["hand_mesh2x1_L2.json", "hand_mesh1x2_L1.json"])
def test_assembly_matches_hand_derived_matrix(name):
    g, p = golden_problem(name)
    J = ops.dense_matrix(p, g["nx"], g["ny"], g["L"])
    assert np.array_equal(J, np.array(g["J"], dtype=float))


@pytest.mark.parametrize("name", ["hand_mesh2x1_L2.json", "hand_mesh1x2_L1.json"])
def test_structured_route_matches_hand_matrix(name):
    g, p = golden_problem(name)
    m = g["L"] + 3
    N = g["nx"] * g["ny"]
    J = np.array(g["J"], dtype=float)
    for j in range(N * m):  # every column of J through the CSR + BR1 route
        e = np.zeros(N * m)
        e[j] = 1.0
        y = formats.structured_matvec(p, g["nx"], g["ny"], g["L"], e)
        assert np.array_equal(y, J[:, j])


SHAPES = [(16, 16, 8), (1, 1, 1), (3, 2, 1), (5, 3, 2), (4, 7, 5), (2, 9, 4)]


@pytest.mark.parametrize("nx,ny,L", SHAPES)
def test_structured_matvec_equals_assembled(nx, ny, L):
    # self-check 1: structured (CSR + block rank-one) product = dense J x
    p = gen.make_problem(nx, ny, L, seed=11)
    x = gen.make_vector(nx, ny, L, seed=2)[0]
    J = ops.dense_matrix(p, nx, ny, L)
    y_dense = J @ x.ravel()
    y_struct = formats.structured_matvec(p, nx, ny, L, x)
    assert rel(y_struct, y_dense) <= 1e-13
    y_bsr = ops.matvec(p, nx, ny, L, x)
    assert rel(y_bsr.ravel(), y_dense) <= 1e-13


@pytest.mark.parametrize("nx,ny,L", [(16, 16, 8), (3, 4, 3)])
def test_bsr_matvec_equals_scipy_bsr(nx, ny, L):
    # the paper's own baseline routine (scipy.sparse.bsr_array.dot, section 5.2)
    p = gen.make_problem(nx, ny, L, seed=4)
    m = L + 3
    indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L)
    A = sp.bsr_array((data, indices, indptr), shape=(nx * ny * m, nx * ny * m))
    x = gen.make_vector(nx, ny, L, nrhs=2, seed=5)
    y = ops.matvec(p, nx, ny, L, x)
    for r in range(2):
        assert rel(y[r].ravel(), A @ x[r].ravel()) <= 1e-14


def test_neighbour_semantics():
    # a vector supported on one cell is seen by the cell north of it through
    # that cell's SOUTH block, by the east cell through its WEST block, ...
    nx, ny, L = 5, 4, 3
    p = gen.make_problem(nx, ny, L, seed=9)
    m = L + 3
    c0 = 2 * nx + 2
    x = np.zeros((nx * ny, m))
    x[c0] = np.random.default_rng(0).standard_normal(m)
    y = ops.matvec(p, nx, ny, L, x)
    touched = {c0 + nx: mesh.S, c0 - nx: mesh.N, c0 + 1: mesh.W, c0 - 1: mesh.E}
    for c, d in touched.items():
        D = np.diag(p["s_nbr"][c, mesh.NBR_SLOT[d]]) + np.outer(p["u"][c, d], p["v"][c, d])
        assert np.allclose(y[c], D @ x[c0], rtol=1e-14, atol=0)
    others = [c for c in range(nx * ny) if c not in touched and c != c0]
    assert np.all(y[others] == 0.0)


def test_generator_zeroes_missing_blocks_and_matvec_ignores_them():
    nx, ny, L = 3, 3, 2
    p = gen.make_problem(nx, ny, L, seed=1)
    ex = gen.block_exists(nx, ny)
    assert not np.any(p["u"][~ex]) and not np.any(p["v"][~ex])
    for j, d in enumerate(gen.NBR_DIRS):
        assert not np.any(p["s_nbr"][~ex[:, d], j])
    assert ex.sum() == 5 * nx * ny - 2 * nx - 2 * ny


@pytest.mark.parametrize("nx,ny,L", [(16, 16, 8), (3, 5, 2), (1, 1, 4)])
def test_transpose_matvec(nx, ny, L):
    p = gen.make_problem(nx, ny, L, seed=3)
    J = ops.dense_matrix(p, nx, ny, L)
    x = gen.make_vector(nx, ny, L, seed=7)[0]
    y = gen.make_vector(nx, ny, L, seed=8)[0]
    jt = ops.matvec_T(p, nx, ny, L, y)
    assert rel(jt.ravel(), J.T @ y.ravel()) <= 1e-13
    lhs = float(np.dot(y.ravel(), ops.matvec(p, nx, ny, L, x).ravel()))
    rhs = float(np.dot(jt.ravel(), x.ravel()))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(J) * np.linalg.norm(x) * np.linalg.norm(y)


def test_matvec_rows_matches_full():
    nx, ny, L = 7, 5, 4
    p = gen.make_problem(nx, ny, L, seed=2)
    x = gen.make_vector(nx, ny, L, nrhs=3, seed=1)
    y = ops.matvec(p, nx, ny, L, x)
    cells = [0, 6, 17, 34, 12]
    yr = ops.matvec_rows(p, nx, ny, L, x, cells)
    assert np.array_equal(yr, y[:, cells, :])


def test_generator_distributions_and_dominance():
    nx, ny, L = 64, 32, 20
    p = gen.make_problem(nx, ny, L, seed=0)
    m = L + 3
    assert np.all(p["s_diag"] >= 20.0)
    # |N(0,1)| has mean sqrt(2/pi)
    assert abs((p["s_diag"] - 20.0).mean() / 10.0 - np.sqrt(2 / np.pi)) < 0.02
    ex = gen.block_exists(nx, ny)
    nb = p["s_nbr"][ex[:, list(gen.NBR_DIRS)]]
    assert nb.min() >= -1.0 and nb.max() <= 0.0 and abs(nb.mean() + 0.5) < 0.01
    uv = p["u"][ex]
    assert abs(uv.std() - 0.1) < 0.002
    # strict row diagonal dominance of S (inv_dt = 20)
    off = np.zeros((nx * ny, m))
    off[:, 1:L] += np.abs(p["s_sub"])
    off[:, :L - 1] += np.abs(p["s_sup"])
    pairs = assemble.FLOW_PAIRS
    for t, (i, j) in enumerate(pairs):
        off[:, L + i] += np.abs(p["s_flow"][:, t])
    off += np.abs(p["s_nbr"]).sum(axis=1)
    assert np.all(p["s_diag"] > off)
    # determinism
    q = gen.make_problem(nx, ny, L, seed=0)
    assert all(np.array_equal(p[k], q[k]) for k in gen.FIELDS)


def test_transpose_rows_match_full_transpose():
    nx, ny, L = 6, 5, 3
    p = gen.make_problem(nx, ny, L, seed=12)
    x = gen.make_vector(nx, ny, L, nrhs=2, seed=3)
    full = ops.matvec_T(p, nx, ny, L, x)
    cells = [0, 5, 7, 14, 29, 24]
    assert np.allclose(ops.matvec_T_rows(p, nx, ny, L, x, cells), full[:, cells], rtol=1e-14,
                       atol=1e-14)
