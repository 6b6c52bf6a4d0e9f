"""GPU parity on general 2-D meshes: the block structure is given by
BR1-BSR style index arrays (section 5.1) instead of the structured stencil.
Unstructured meshes are Delaunay triangulations of random points (every
triangle a cell, at most three neighbours), cell numbering shuffled.  Checks
against the general-mesh oracle (dense blocks, dense LU)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, U32, block_jacobi_ref, check_componentwise, host, log, relnorm, vec
from oracle import blockjacobi, graph, ops
from paper_2403_09198_amd import gen, r1s

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def graph_dev(p):
    keys = gen.GRAPH_FIELDS + tuple(k for k in gen.PATTERN_FIELDS if k in p)
    return {k: torch.from_numpy(np.ascontiguousarray(p[k])).to(DEV) for k in keys}


def _setup(ip, ix, L, ranks=(1, 1), band=1, arrow=False, seed=1, keep_f32=True,
           with_trans=True):
    p = gen.make_graph_problem(ip, ix, L, seed=seed, r_diag=ranks[0], r_off=ranks[1], band=band,
                               arrow=arrow)
    A = r1s.R1GraphMatrix(ip, ix, L, graph_dev(p), keep_f32=keep_f32, ranks=ranks, band=band,
                          arrow=arrow)
    M = r1s.SMWPreconditioner(A, keep_f32=keep_f32, with_trans=with_trans)
    return p, A, M


def _scale(p, L, x, trans=False, cells=None):
    pa = graph.abs_problem(p)
    if cells is None:
        return (graph.matvec_T if trans else graph.matvec)(pa, L, np.abs(x))
    return (graph.matvec_T_rows if trans else graph.matvec_rows)(pa, L, np.abs(x), cells)


def _bj_ref(p, L, r, cells=None, trans=False):
    N = len(p["graph_indptr"]) - 1
    cells = list(range(N)) if cells is None else cells
    LU, piv = blockjacobi.lu_factor(graph.diagonal_blocks(p, L, cells))
    f = blockjacobi.lu_solve_T if trans else blockjacobi.lu_solve
    return np.stack([f(LU, piv, r[i][cells]) for i in range(r.shape[0])])


def _per_cell_rel(z, ref):
    num = np.linalg.norm(z - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float(np.max(num / den))


CASES = [(40, 8, (1, 1), 1, False), (25, 61, (9, 2), 1, False), (30, 62, (3, 1), 3, True),
         (12, 200, (1, 2), 2, False), (6, 1, (2, 0), 1, False), (50, 6, (9, 2), 4, True)]


@pytest.mark.parametrize("npts,L,ranks,band,arrow", CASES)
def test_delaunay_parity(npts, L, ranks, band, arrow):
    log(f"delaunay parity npts={npts} L={L} ranks={ranks} band={band} arrow={arrow}")
    ip, ix = gen.delaunay_graph(npts, seed=npts)
    p, A, M = _setup(ip, ix, L, ranks, band, arrow)
    N, m = len(ip) - 1, L + 3
    P = ranks[0] + 3 * ranks[1]
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, N, m))
    xd = vec(x)
    ref, reft = graph.matvec(p, L, x), graph.matvec_T(p, L, x)
    sc, sct = _scale(p, L, x), _scale(p, L, x, trans=True)
    check_componentwise(host(A.matvec(xd)), ref, sc, TOL64, "J x")
    check_componentwise(host(A.matvec(xd, trans=True)), reft, sct, TOL64, "J^T x")
    tol32 = (m + P + 2 * band + 16) * U32
    check_componentwise(host(A.matvec(xd, precision="f32")), ref, sc, tol32, "J x (f32)")
    check_componentwise(host(A.matvec(xd, trans=True, precision="f32")), reft, sct, tol32,
                        "J^T x (f32)")
    b = rng.standard_normal((3, N, m))
    check_componentwise(host(A.residual(vec(b), xd)), b - ref, sc + np.abs(b), TOL64, "b - J x")
    r = rng.standard_normal((3, N, m))
    rd = vec(r)
    assert _per_cell_rel(host(M.apply(rd)), _bj_ref(p, L, r)) <= TOL64
    assert _per_cell_rel(host(M.apply(rd, trans=True)), _bj_ref(p, L, r, trans=True)) <= TOL64


def test_structured_mesh_as_graph_matches_structured_path():
    nx, ny, L = 9, 7, 61
    log("structured mesh through the general-mesh path")
    p = gen.make_problem(nx, ny, L, seed=2, r_diag=9, r_off=2)
    q = gen.graph_from_structured(p, nx, ny)
    ip, ix = q["graph_indptr"], q["graph_indices"]
    A = r1s.R1GraphMatrix(ip, ix, L, graph_dev(q), ranks=(9, 2))
    from gpu_util import to_dev
    S = r1s.R1Matrix(nx, ny, L, to_dev(p), ranks=(9, 2))
    x = vec(gen.make_vector(nx, ny, L, nrhs=2, seed=3))
    for tr in (False, True):
        a, s = host(A.matvec(x, trans=tr)), host(S.matvec(x, trans=tr))
        assert relnorm(a, s) <= 1e-14, tr
    # same stored values; the general mesh adds only its slot tables
    sa, ss = A.storage(), S.storage()
    assert sa["structured_values"] == ss["structured_values"]
    assert sa["index_bytes"] == 4 * (2 * nx * ny * 4 + nx * ny)


def test_gmres_bsr_and_gradients_on_delaunay():
    ip, ix = gen.delaunay_graph(120, seed=11)
    L = 8
    log("delaunay gmres / bsr / gradients")
    p, A, M = _setup(ip, ix, L, (9, 2), 2, True, seed=3)
    N, m = len(ip) - 1, L + 3
    rng = np.random.default_rng(5)
    b = rng.standard_normal((2, N, m))
    J = graph.dense_matrix(p, L)
    for kw in (dict(), dict(trans=True), dict(mode="mixed")):
        res = r1s.gmres(A, M, vec(b), restart=30, rtol=1e-12, **kw)
        Jm = J.T if kw.get("trans") else J
        for r in range(2):
            assert res.stats[r]["converged"] == 1, kw
            assert relnorm(host(res.x)[r].ravel(), np.linalg.solve(Jm, b[r].ravel())) <= 1e-10, kw
    B = r1s.BSRMatrix(A)
    Pl = r1s.DenseLUPreconditioner(B)
    x = rng.standard_normal((2, N, m))
    check_componentwise(host(B.matvec(vec(x))), graph.matvec(p, L, x), _scale(p, L, x), TOL64,
                        "BSR J x")
    assert _per_cell_rel(host(Pl.apply(vec(x))), _bj_ref(p, L, x)) <= TOL64
    rb = r1s.gmres(A, Pl, vec(b), restart=30, rtol=1e-12, op="bsr", B=B)
    assert relnorm(host(rb.x)[0].ravel(), np.linalg.solve(J, b[0].ravel())) <= 1e-10
    lam = rng.standard_normal((3, N, m))
    xx = rng.standard_normal((3, N, m))
    g = r1s.grad(A, vec(lam), vec(xx))
    ref = graph.grads(p, L, lam, xx)
    for k in g:
        assert relnorm(host(g[k]), ref[k]) <= 1e-13, k


def test_full_size_delaunay_sampled_parity():
    # about 32 000 triangle cells, L = 61, the paper's pair counts
    L = 61
    log("full-size delaunay sampled parity")
    ip, ix = gen.delaunay_graph(16400, seed=1)
    p, A, M = _setup(ip, ix, L, gen.PAPER_RANKS, seed=0, keep_f32=False)
    N, m = len(ip) - 1, L + 3
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, N, m))
    xd = vec(x)
    cells = sorted(set(rng.choice(N, 40, replace=False).tolist()) | {0, N - 1})
    check_componentwise(host(A.matvec(xd))[:, cells], graph.matvec_rows(p, L, x, cells),
                        _scale(p, L, x, cells=cells), TOL64, "J x sampled")
    check_componentwise(host(A.matvec(xd, trans=True))[:, cells],
                        graph.matvec_T_rows(p, L, x, cells),
                        _scale(p, L, x, trans=True, cells=cells), TOL64, "J^T x sampled")
    assert _per_cell_rel(host(M.apply(xd))[:, cells], _bj_ref(p, L, x, cells)) <= TOL64
    w = vec(rng.standard_normal((1, N, m)))
    lhs = float(torch.dot(w.ravel(), A.matvec(xd).ravel()))
    rhs = float(torch.dot(A.matvec(w, trans=True).ravel(), xd.ravel()))
    scale = float(torch.linalg.norm(w)) * float(torch.linalg.norm(xd))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + scale)


def test_general_mesh_errors():
    ip, ix = gen.delaunay_graph(20, seed=3)
    L = 4
    p = gen.make_graph_problem(ip, ix, L, seed=1)
    vals = graph_dev(p)
    with pytest.raises(ValueError):
        r1s.R1GraphMatrix(ip, ix, L, vals, ranks=(2, 1))  # u_diag holds one pair
    A = r1s.R1GraphMatrix(ip, ix, L, vals)
    z = vec(np.zeros((1, len(ip) - 1, L + 3)))
    # the structured-mesh gradient call refuses a general-mesh handle
    with pytest.raises(r1s.R1SError):
        r1s.r1s_grad(A.h, 1, z, z, {})
