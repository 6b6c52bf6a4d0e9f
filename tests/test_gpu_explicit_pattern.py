"""GPU parity with a general pattern of the diagonal block shared by every
cell (section 4, "Temporal Source Jacobian": the nonzeros of S_cc follow
from the kinetic processes kept).  The library analyses the pattern once on
the host (ELL rows and dense indices for the products; minimum-degree order
and the fill of LU without pivoting for the block-Jacobi) and every cell
follows the same tables.  All checks against the CPU oracle: dense blocks,
dense LU, the dense-block chain rule for gradients."""
import numpy as np
import pytest
import torch

from gpu_util import (DEV, U32, block_jacobi_ref, check_componentwise, host, log, matvec_scale,
                      relnorm, sample_cells, vec)
from oracle import assemble, grads as ograds, ops
from paper_2403_09198_amd import gen, r1s
from paper_2403_09198_amd._lib import R1S_ERR_SINGULAR

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _dev(p):
    return {k: torch.from_numpy(np.ascontiguousarray(p[k])).to(DEV)
            for k in gen.PATTERN_PROBLEM_FIELDS}


def _pattern(m, kind, seed):
    if kind == "random":
        return gen.random_pattern(m, per_row=3, dense_rows=(m // 2,), dense_cols=(1,), seed=seed)
    if kind == "sparse":
        return gen.random_pattern(m, per_row=2, seed=seed)
    if kind == "wide":  # rows and columns of up to 12 entries, no dense index needed
        return gen.random_pattern(m, per_row=min(m - 1, 10), seed=seed)
    L = m - 3
    band, arrow = {"band3": (3, 0), "arrow": (1, 1), "atom": (2, 2)}[kind]
    return gen.layout_pattern(L, band, arrow)


def _setup(nx, ny, L, kind, ranks=(1, 1), seed=1, keep_f32=True, with_trans=True):
    ip, ix = _pattern(L + 3, kind, seed)
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=seed, r_diag=ranks[0], r_off=ranks[1])
    A = r1s.R1PatternMatrix(nx, ny, L, (ip, ix), _dev(p), keep_f32=keep_f32, ranks=ranks)
    M = r1s.SMWPreconditioner(A, keep_f32=keep_f32, with_trans=with_trans)
    return p, A, M


def _per_cell_rel(z, ref):
    num = np.linalg.norm(z - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float(np.max(num / den))


SHAPES = [(5, 3, 8), (1, 1, 1), (3, 4, 61), (2, 3, 62), (2, 2, 125), (2, 2, 200), (70, 2, 6)]
KINDS = ["random", "sparse", "wide", "band3", "arrow", "atom"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("nx,ny,L", SHAPES)
@pytest.mark.parametrize("ranks", [(1, 1), (9, 2), (2, 6)], ids=lambda r: f"r{r[0]}_{r[1]}")
def test_pattern_matvec_and_smw_parity(nx, ny, L, kind, ranks):
    if kind in ("atom", "arrow", "band3") and L < 2:
        pytest.skip("layout patterns need molecule levels")
    log(f"explicit pattern {kind} ranks={ranks} nx={nx} ny={ny} L={L}")
    p, A, M = _setup(nx, ny, L, kind, ranks)
    m, P = L + 3, ranks[0] + 4 * ranks[1]
    nnz_row = int(np.max(np.diff(p["pat_indptr"])))
    x = gen.make_vector(nx, ny, L, nrhs=3, seed=4)
    xd = vec(x)
    ref, reft = ops.matvec(p, nx, ny, L, x), ops.matvec_T(p, nx, ny, L, x)
    sc, sct = matvec_scale(p, nx, ny, L, x), matvec_scale(p, nx, ny, L, x, trans=True)
    check_componentwise(host(A.matvec(xd)), ref, sc, TOL64, "J x")
    check_componentwise(host(A.matvec(xd, trans=True)), reft, sct, TOL64, "J^T x")
    # float32: a row or column holds at most nnz_row + 4 + P products
    tol32 = (nnz_row + m + P + 16) * U32
    check_componentwise(host(A.matvec(xd, precision="f32")), ref, sc, tol32, "J x (f32)")
    check_componentwise(host(A.matvec(xd, trans=True, precision="f32")), reft, sct, tol32,
                        "J^T x (f32)")
    b = gen.make_rhs(nx, ny, L, nrhs=3, seed=4)
    check_componentwise(host(A.residual(vec(b), xd)), b - ref, sc + np.abs(b), TOL64, "b - J x")
    r = gen.make_rhs(nx, ny, L, nrhs=3, seed=6)
    rd = vec(r)
    zref = block_jacobi_ref(p, nx, ny, L, r)
    zreft = block_jacobi_ref(p, nx, ny, L, r, trans=True)
    assert _per_cell_rel(host(M.apply(rd)), zref) <= TOL64
    assert _per_cell_rel(host(M.apply(rd, trans=True)), zreft) <= TOL64
    tol32s = 8 * (m * 4 + ranks[0] ** 2) * U32
    assert _per_cell_rel(host(M.apply(rd, precision="f32")), zref) <= tol32s
    assert _per_cell_rel(host(M.apply(rd, trans=True, precision="f32")), zreft) <= tol32s


@pytest.mark.parametrize("band,arrow", [(1, 0), (3, 0), (1, 1), (4, 1), (1, 2), (3, 2)])
def test_layout_pattern_matches_the_structured_path(band, arrow):
    # the same Jacobian once through a structured layout, once as an explicit
    # pattern: the two library paths agree to rounding
    nx, ny, L = 6, 5, 20
    log(f"explicit pattern vs structured band={band} arrow={arrow}")
    q = gen.make_problem(nx, ny, L, seed=3, band=band, arrow=arrow, r_diag=2, r_off=1)
    ip, ix = gen.layout_pattern(L, band, arrow)
    row = np.repeat(np.arange(L + 3), np.diff(ip))
    blocks = [assemble.diagonal_sparse_block(q, c, L) for c in range(nx * ny)]
    p = {"pat_indptr": ip, "pat_indices": ix, "ranks": q["ranks"],
         "s_cc": np.stack([B[row, ix] for B in blocks]), "s_nbr": q["s_nbr"], "u": q["u"],
         "v": q["v"]}
    keys = gen.FIELDS + tuple(k for k in gen.PATTERN_FIELDS if k in q)
    As = r1s.R1Matrix(nx, ny, L, {k: vec(q[k]) for k in keys}, ranks=(2, 1), band=band,
                      arrow=arrow)
    Ms = r1s.SMWPreconditioner(As, with_trans=True)
    Ap = r1s.R1PatternMatrix(nx, ny, L, (ip, ix), _dev(p), ranks=(2, 1))
    Mp = r1s.SMWPreconditioner(Ap, with_trans=True)
    x = gen.make_vector(nx, ny, L, nrhs=2, seed=2)
    xd = vec(x)
    for tr in (False, True):
        sc = matvec_scale(q, nx, ny, L, x, trans=tr)
        check_componentwise(host(Ap.matvec(xd, trans=tr)), host(As.matvec(xd, trans=tr)), sc,
                            2 * TOL64, f"pattern vs structured (trans {tr})")
        assert _per_cell_rel(host(Mp.apply(xd, trans=tr)), host(Ms.apply(xd, trans=tr))) <= 2 * TOL64


@pytest.mark.parametrize("kind", ["random", "atom"])
def test_pattern_gmres(kind):
    nx, ny, L = 12, 10, 13
    log(f"explicit pattern gmres {kind}")
    p, A, M = _setup(nx, ny, L, kind, gen.PAPER_RANKS, seed=3)
    b = gen.make_rhs(nx, ny, L, nrhs=2, seed=3)
    J = ops.dense_matrix(p, nx, ny, L)
    for kw in (dict(), dict(trans=True), dict(mode="mixed")):
        res = r1s.gmres(A, M, vec(b), restart=30, rtol=1e-12, **kw)
        Jm = J.T if kw.get("trans") else J
        for r in range(2):
            assert res.stats[r]["converged"] == 1, kw
            assert relnorm(host(res.x)[r].ravel(), np.linalg.solve(Jm, b[r].ravel())) <= 1e-10, kw


@pytest.mark.parametrize("kind", ["random", "atom", "wide"])
def test_pattern_grad_kernel_matches_oracle(kind):
    nx, ny, L, nrhs = 5, 4, 9, 3
    log(f"explicit pattern grad {kind}")
    p, A, M = _setup(nx, ny, L, kind, (2, 1), seed=4, keep_f32=False, with_trans=False)
    lam = gen.make_vector(nx, ny, L, nrhs=nrhs, seed=5)
    x = gen.make_vector(nx, ny, L, nrhs=nrhs, seed=6)
    g = r1s.grad(A, vec(lam), vec(x))
    ref = ograds.structured_grads(p, nx, ny, L, lam, x)
    assert set(g) == set(ref)
    for k in g:
        assert relnorm(host(g[k]), ref[k]) <= 1e-13, k


@pytest.mark.parametrize("nx,ny,L", [(6, 5, 8), (3, 4, 62)])
def test_pattern_bsr_parity(nx, ny, L):
    log(f"explicit pattern bsr nx={nx} ny={ny} L={L}")
    p, A, M = _setup(nx, ny, L, "random", (9, 2), keep_f32=False, with_trans=False)
    B = r1s.BSRMatrix(A)
    Pl = r1s.DenseLUPreconditioner(B)
    x = gen.make_vector(nx, ny, L, nrhs=2, seed=9)
    xd = vec(x)
    check_componentwise(host(B.matvec(xd)), ops.matvec(p, nx, ny, L, x),
                        matvec_scale(p, nx, ny, L, x), TOL64, "BSR J x")
    assert _per_cell_rel(host(Pl.apply(xd)), block_jacobi_ref(p, nx, ny, L, x)) <= TOL64


def test_pattern_update_and_full_size_sampled_parity():
    nx, ny, L = 256, 128, 61
    log("explicit pattern full size 256x128 L=61 (atom layout pattern, ranks (9, 2))")
    ip, ix = gen.layout_pattern(L, 2, 2)
    p0 = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=1, r_diag=9, r_off=2)
    A = r1s.R1PatternMatrix(nx, ny, L, (ip, ix), _dev(p0), ranks=(9, 2))
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=0, r_diag=9, r_off=2)
    A.update(_dev(p))
    M = r1s.SMWPreconditioner(A, with_trans=True)
    x = gen.make_vector(nx, ny, L, seed=0)
    xd = vec(x)
    cells = sample_cells(nx, ny)
    check_componentwise(host(A.matvec(xd))[:, cells], ops.matvec_rows(p, nx, ny, L, x, cells),
                        matvec_scale(p, nx, ny, L, x, cells), TOL64, "J x sampled")
    check_componentwise(host(A.matvec(xd, trans=True))[:, cells],
                        ops.matvec_T_rows(p, nx, ny, L, x, cells),
                        matvec_scale(p, nx, ny, L, x, cells, trans=True), TOL64, "J^T x sampled")
    assert _per_cell_rel(host(M.apply(xd))[:, cells], block_jacobi_ref(p, nx, ny, L, x, cells)) \
        <= TOL64
    assert _per_cell_rel(host(M.apply(xd, trans=True))[:, cells],
                         block_jacobi_ref(p, nx, ny, L, x, cells, trans=True)) <= TOL64


def test_pattern_zero_row_is_reported():
    nx, ny, L = 4, 3, 6
    ip, ix = gen.random_pattern(L + 3, per_row=2, seed=2)
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=2)
    c, i = 7, 4
    p["s_cc"][c, ip[i]:ip[i + 1]] = 0.0  # row i of S_cc is zero
    p["u"][c, :, i] = 0.0
    A = r1s.R1PatternMatrix(nx, ny, L, (ip, ix), _dev(p))
    with pytest.raises(r1s.R1SError) as ei:
        r1s.SMWPreconditioner(A)
    assert ei.value.code == R1S_ERR_SINGULAR and "cell 7" in str(ei.value)


def test_pattern_storage_counts():
    nx, ny, L = 3, 2, 9
    ip, ix = gen.random_pattern(L + 3, per_row=3, seed=0)
    p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=0, r_diag=2, r_off=1)
    A = r1s.R1PatternMatrix(nx, ny, L, (ip, ix), _dev(p), ranks=(2, 1))
    from oracle import storage
    assert A.storage()["structured_values"] == storage.explicit_pattern_values(
        nx, ny, L + 3, len(ix), 2, 1)
