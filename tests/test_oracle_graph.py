"""Pins of the general-mesh oracle (block structure from the BR1-BSR index
arrays of section 5.1): the structured mesh written as a graph reproduces
the structured oracle, the dense-block product equals the CSR + BR1 product
of section 5.2 on unstructured (Delaunay) meshes, and the solver pieces hold
their identities there."""
import numpy as np
import pytest

from conftest import rel
from oracle import assemble, blockjacobi, formats, gmres, graph, grads, mesh, ops
from paper_2403_09198_amd import gen


@pytest.mark.parametrize("ranks,band,arrow", [((1, 1), 1, False), ((9, 2), 3, True),
                                              ((2, 0), 2, False), ((2, 1), 2, 2)])
def test_structured_mesh_as_graph_matches_structured_oracle(ranks, band, arrow):
    nx, ny, L = 5, 4, 7
    p = gen.make_problem(nx, ny, L, seed=3, r_diag=ranks[0], r_off=ranks[1], band=band,
                         arrow=arrow)
    q = gen.graph_from_structured(p, nx, ny)
    x = gen.make_vector(nx, ny, L, nrhs=2, seed=1)
    assert rel(graph.matvec(q, L, x), ops.matvec(p, nx, ny, L, x)) <= 1e-14
    assert rel(graph.matvec_T(q, L, x), ops.matvec_T(p, nx, ny, L, x)) <= 1e-14
    assert rel(graph.dense_matrix(q, L), ops.dense_matrix(p, nx, ny, L)) <= 1e-15


@pytest.mark.parametrize("ranks,band,arrow", [((1, 1), 1, False), ((9, 2), 4, True),
                                              ((3, 1), 1, True), ((2, 1), 1, 2)])
def test_delaunay_dense_product_equals_csr_plus_br1(ranks, band, arrow):
    indptr, indices = gen.delaunay_graph(60, seed=4)
    L = 6
    p = gen.make_graph_problem(indptr, indices, L, seed=5, r_diag=ranks[0], r_off=ranks[1],
                               band=band, arrow=arrow)
    N = len(indptr) - 1
    x = np.random.default_rng(0).standard_normal((N, L + 3))
    assert rel(graph.matvec(p, L, x).ravel(), formats.graph_matvec(p, L, x)) <= 1e-13
    J = graph.dense_matrix(p, L)
    assert rel(J @ x.ravel(), formats.graph_matvec(p, L, x)) <= 1e-13
    w = np.random.default_rng(1).standard_normal((N, L + 3))
    assert abs(np.vdot(w, graph.matvec(p, L, x)) - np.vdot(graph.matvec_T(p, L, w), x)) <= \
        1e-12 * np.linalg.norm(w) * np.linalg.norm(x) * np.abs(J).max()


def test_delaunay_mesh_structure():
    indptr, indices = gen.delaunay_graph(300, seed=2)
    N = len(indptr) - 1
    deg = np.diff(indptr) - 1
    assert deg.max() <= 3 and deg.min() >= 1
    # structurally symmetric, diagonal once per row
    pairs = set()
    for c in range(N):
        row = indices[indptr[c]:indptr[c + 1]]
        assert list(row).count(c) == 1
        pairs |= {(c, int(j)) for j in row if j != c}
    assert all((j, c) in pairs for c, j in pairs)
    # Euler's formula for a triangulation of a convex hull: interior edges
    n_int_edges = len(pairs) // 2
    assert 3 * N == 2 * n_int_edges + int(np.sum(3 - deg))


@pytest.mark.parametrize("r_diag", [1, 9])
def test_woodbury_inverse_on_graph_cells(r_diag):
    indptr, indices = gen.delaunay_graph(30, seed=7)
    L = 12
    p = gen.make_graph_problem(indptr, indices, L, seed=8, r_diag=r_diag, r_off=2, band=2,
                               arrow=True)
    v = graph.smw_view(p)
    for c in range(len(indptr) - 1):
        D = graph.diag_block(p, c, L)
        assert np.abs(blockjacobi.smw_inverse(v, c, L) @ D - np.eye(L + 3)).max() <= 1e-12


def test_gmres_on_delaunay_mesh_matches_dense_solve():
    indptr, indices = gen.delaunay_graph(80, seed=9)
    L = 5
    p = gen.make_graph_problem(indptr, indices, L, seed=9, r_diag=9, r_off=2)
    N = len(indptr) - 1
    b = np.random.default_rng(3).standard_normal((N, L + 3))
    BJ = blockjacobi.BlockJacobi(graph.diagonal_blocks(p, L))
    res = gmres.gmres(lambda v: graph.matvec(p, L, v), BJ.apply, b, restart=30, rtol=1e-12)
    J = graph.dense_matrix(p, L)
    assert res.converged
    assert rel(res.x.ravel(), np.linalg.solve(J, b.ravel())) <= 2 * np.linalg.cond(J) * 1e-12


def test_storage_counts_on_graph():
    indptr, indices = gen.delaunay_graph(50, seed=1)
    L = 7
    for ranks, band, arrow in (((1, 1), 1, False), ((9, 2), 3, True), ((2, 1), 2, 2)):
        p = gen.make_graph_problem(indptr, indices, L, seed=1, r_diag=ranks[0], r_off=ranks[1],
                                   band=band, arrow=arrow)
        csr = formats.graph_csr(p, L)
        br1 = formats.graph_br1(p)
        counted = csr[0].size + br1["column_data"].size + br1["row_data"].size
        assert graph.structured_values(p, L) == counted


def test_graph_gradients_match_finite_differences():
    indptr, indices = gen.delaunay_graph(12, seed=3)
    L, nrhs = 4, 2
    p = gen.make_graph_problem(indptr, indices, L, seed=4, r_diag=2, r_off=1, band=2, arrow=True)
    N = len(indptr) - 1
    n = N * (L + 3)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((nrhs, N, L + 3))
    w = rng.standard_normal((nrhs, N, L + 3))

    def loss_of(q):
        J = graph.dense_matrix(q, L)
        return grads.loss(np.linalg.solve(J, b.reshape(nrhs, n).T).T, w.reshape(nrhs, n))

    J = graph.dense_matrix(p, L)
    x = np.linalg.solve(J, b.reshape(nrhs, n).T).T.reshape(b.shape)
    lam = np.linalg.solve(J.T, w.reshape(nrhs, n).T).T.reshape(b.shape)
    g = graph.grads(p, L, lam, x)
    h = 1e-6
    for key in g:
        for _ in range(4):
            idx = tuple(int(rng.integers(s)) for s in p[key].shape)
            qp = {kk: vv.copy() for kk, vv in p.items()}
            qm = {kk: vv.copy() for kk, vv in p.items()}
            qp[key][idx] += h
            qm[key][idx] -= h
            fd = (loss_of(qp) - loss_of(qm)) / (2 * h)
            assert abs(fd - g[key][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, idx)
