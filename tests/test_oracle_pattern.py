"""Pins of the oracle with a wider diagonal sparse block.

Section 4 ("Temporal Source Jacobian"): level-changing processes up to a
threshold jump in the level index give a banded pattern whose width is set by
that threshold, and the level sources also depend on the temperature, so the
level rows see the flow unknowns.  The generator's `band` is the band
half-width over the levels (1 = tridiagonal) and `arrow` adds level/flow
coupling (level rows x flow columns and flow rows x level columns); arrow = 2
also couples the last level, the atom density, to every molecule level (the
DRa processes of the same passage: a dense atom column and atom row)."""
import numpy as np
import pytest
from scipy.linalg import solve_banded

from conftest import rel
from oracle import assemble, blockjacobi, formats, gmres, grads, mesh, ops, storage
from paper_2403_09198_amd import gen

PATTERNS = [(2, False), (3, True), (4, False), (1, True), (4, True), (1, 2), (3, 2)]


@pytest.mark.parametrize("band,arrow", PATTERNS)
def test_structured_product_equals_assembled(band, arrow):
    nx, ny, L = 4, 3, 9
    p = gen.make_problem(nx, ny, L, seed=11, band=band, arrow=arrow, r_diag=2, r_off=1)
    x = gen.make_vector(nx, ny, L, seed=3)[0]
    J = ops.dense_matrix(p, nx, ny, L)
    assert rel(formats.structured_matvec(p, nx, ny, L, x), J @ x.ravel()) <= 1e-13
    assert rel(ops.matvec(p, nx, ny, L, x).ravel(), J @ x.ravel()) <= 1e-13
    assert rel(ops.matvec_T(p, nx, ny, L, x).ravel(), J.T @ x.ravel()) <= 1e-13


@pytest.mark.parametrize("band", [2, 3, 5])
def test_band_orientation_against_banded_solver(band):
    # without coupling the level block is banded: LAPACK's banded solver on
    # the diagonal-ordered storage built straight from the input arrays
    L = 12
    p = gen.make_problem(2, 1, L, seed=5, band=band, arrow=False)
    c = 1
    ab = np.zeros((2 * band + 1, L))
    ab[band] = p["s_diag"][c, :L]
    ab[band - 1, 1:] = p["s_sup"][c]           # S[k][k+1] sits at column k+1
    ab[band + 1, :-1] = p["s_sub"][c]          # S[k+1][k] sits at column k
    for j in range(2, band + 1):
        ab[band - j, j:] = p["s_band"][c, band - 1 + j - 2, :L - j]   # S[k][k+j]
        ab[band + j, :L - j] = p["s_band"][c, j - 2, j:]             # S[k][k-j]
    r = gen.make_vector(2, 1, L, seed=1)[0, c]
    x = blockjacobi.sparse_diag_solve(p, c, L, r)
    assert rel(x[:L], solve_banded((band, band), ab, r[:L])) <= 1e-13
    # and the flow corner stays uncoupled
    assert rel(x[L:], np.linalg.solve(assemble.diagonal_sparse_block(p, c, L)[L:, L:], r[L:])) <= 1e-13


def test_arrow_entries_sit_in_level_flow_positions():
    L = 5
    p = gen.make_problem(1, 1, L, seed=2, band=1, arrow=True)
    A = assemble.diagonal_sparse_block(p, 0, L)
    for i in range(3):
        assert np.array_equal(A[:L, L + i], p["s_lev_flow"][0, i])
        assert np.array_equal(A[L + i, :L], p["s_flow_lev"][0, i])
    # zeroing the coupling gives back the plain pattern
    q = {k: v.copy() for k, v in p.items()}
    q["s_lev_flow"][:] = 0.0
    q["s_flow_lev"][:] = 0.0
    plain = {k: v for k, v in q.items() if k not in gen.PATTERN_FIELDS + ("pattern",)}
    assert np.array_equal(assemble.diagonal_sparse_block(q, 0, L),
                          assemble.diagonal_sparse_block(plain, 0, L))


@pytest.mark.parametrize("band", [1, 3])
def test_atom_entries_sit_in_atom_column_and_row(band):
    L = 7
    a = L - 1
    p = gen.make_problem(1, 1, L, seed=2, band=band, arrow=2)
    A = assemble.diagonal_sparse_block(p, 0, L)
    assert np.array_equal(A[:a, a], p["s_lev_flow"][0, 3, :a])
    assert np.array_equal(A[a, :a], p["s_flow_lev"][0, 3, :a])
    assert A[a, a] == p["s_diag"][0, a]
    # the atom keeps its flow couplings from the three flow slots
    for i in range(3):
        assert np.array_equal(A[:L, L + i], p["s_lev_flow"][0, i])
        assert np.array_equal(A[L + i, :L], p["s_flow_lev"][0, i])
    # index a of the atom slot is not an entry
    q = {k: v.copy() for k, v in p.items()}
    q["s_lev_flow"][0, 3, a] = 7.0
    q["s_flow_lev"][0, 3, a] = -7.0
    assert np.array_equal(assemble.diagonal_sparse_block(q, 0, L), A)
    # a band entry that reaches the atom adds to the atom column (the block
    # is the sum of its parts); the generator draws those as zero
    assert p["s_sup"][0, a - 1] == 0.0 and p["s_sub"][0, a - 1] == 0.0
    q["s_sup"][0, a - 1] = 0.5
    assert assemble.diagonal_sparse_block(q, 0, L)[a - 1, a] == 0.5 + p["s_lev_flow"][0, 3, a - 1]
    # clearing the atom slot gives the arrow = 1 block of the same draw
    q = {k: v.copy() for k, v in p.items()}
    q["s_lev_flow"] = q["s_lev_flow"][:, :3].copy()
    q["s_flow_lev"] = q["s_flow_lev"][:, :3].copy()
    q["pattern"] = np.array([band, 1])
    B = assemble.diagonal_sparse_block(q, 0, L)
    assert np.array_equal(B[:a, a], np.zeros(a)) and np.array_equal(B[a, :a], np.zeros(a))
    C = A.copy()
    C[:a, a] = 0.0
    C[a, :a] = 0.0
    assert np.array_equal(C, B)


def test_atom_pattern_counts_per_row():
    # molecule rows: own density, the atom density and the three flow
    # unknowns (plus the band); the atom row: every level and the flow
    L = 9
    a = L - 1
    p = gen.make_problem(1, 1, L, seed=3, band=1, arrow=2)
    q = {k: v.copy() for k, v in p.items()}
    q["s_sub"][:] = 0.0
    q["s_sup"][:] = 0.0
    A = assemble.diagonal_sparse_block(q, 0, L)
    for k in range(a):
        assert set(np.flatnonzero(A[k])) == {k, a, L, L + 1, L + 2}
    assert set(np.flatnonzero(A[a])) == set(range(L + 3))


@pytest.mark.parametrize("band,arrow", PATTERNS)
@pytest.mark.parametrize("r_diag", [1, 9])
def test_woodbury_inverse_times_block_is_identity(band, arrow, r_diag):
    nx, ny, L = 3, 2, 14
    p = gen.make_problem(nx, ny, L, seed=6, band=band, arrow=arrow, r_diag=r_diag, r_off=2)
    for c in range(nx * ny):
        D = assemble.dense_block(p, c, mesh.C, L)
        assert np.abs(blockjacobi.smw_inverse(p, c, L) @ D - np.eye(L + 3)).max() <= 1e-12


def test_gmres_with_wide_pattern_matches_dense_solve():
    nx, ny, L = 6, 5, 10
    p = gen.make_problem(nx, ny, L, seed=8, band=3, arrow=True, r_diag=9, r_off=2)
    b = gen.make_rhs(nx, ny, L, seed=8)[0]
    M = blockjacobi.BlockJacobi(assemble.diagonal_blocks(p, nx, ny, L))
    res = gmres.gmres(lambda v: ops.matvec(p, nx, ny, L, v), M.apply, b, restart=30, rtol=1e-12)
    J = ops.dense_matrix(p, nx, ny, L)
    assert res.converged
    assert rel(res.x.ravel(), np.linalg.solve(J, b.ravel())) <= 2 * np.linalg.cond(J) * 1e-12


def test_storage_counts_with_wide_pattern():
    nx, ny, L = 5, 4, 8
    m = L + 3
    for band, arrow in PATTERNS:
        p = gen.make_problem(nx, ny, L, seed=1, band=band, arrow=arrow, r_diag=3, r_off=1)
        csr = formats.structured_csr(p, nx, ny, L)
        br1 = formats.structured_br1(p, nx, ny)
        counted = csr[0].size + br1["column_data"].size + br1["row_data"].size
        assert storage.structured_values(nx, ny, m, 3, 1, band, arrow) == counted
        # affine in m at a fixed band: zero second difference
        s = [storage.structured_values(nx, ny, mm, 3, 1, band, arrow) for mm in (m - 1, m, m + 1)]
        assert s[2] - 2 * s[1] + s[0] == 0


@pytest.mark.parametrize("arrow", [True, 2])
def test_generator_keeps_dominance_with_wide_pattern(arrow):
    nx, ny, L = 8, 8, 200
    p = gen.make_problem(nx, ny, L, seed=0, band=4, arrow=arrow)
    for c in (0, 9, 27, 63):
        A = assemble.diagonal_sparse_block(p, c, L)
        off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
        nbr = np.abs(p["s_nbr"][c]).sum(axis=0)
        assert np.all(np.abs(np.diag(A)) > off + nbr)


@pytest.mark.parametrize("arrow", [True, 2])
def test_gradients_with_wide_pattern_match_finite_differences(arrow):
    nx, ny, L, nrhs = 3, 2, 6, 2
    p = gen.make_problem(nx, ny, L, seed=4, band=3, arrow=arrow, r_diag=2, r_off=1)
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
    rng = np.random.default_rng(3)
    h = 1e-6
    picks = {k: [tuple(int(rng.integers(s)) for s in p[k].shape) for _ in range(6)]
             for k in gen.PATTERN_FIELDS}
    if arrow == 2:
        a = L - 1
        # every atom-slot entry, its unused index a, and a band entry that
        # reaches the atom (drawn as zero, still a parameter of the sum)
        picks["s_lev_flow"] += [(1, 3, k) for k in range(L)]
        picks["s_flow_lev"] += [(4, 3, k) for k in range(L)]
        picks["s_band"] += [(2, 0, a), (2, 2, a - 3)]
    for key in gen.PATTERN_FIELDS:
        for idx in picks[key]:
            qp = {kk: vv.copy() for kk, vv in p.items()}
            qm = {kk: vv.copy() for kk, vv in p.items()}
            qp[key][idx] += h
            qm[key][idx] -= h
            fd = (loss_of(qp) - loss_of(qm)) / (2 * h)
            # entries outside the band carry no matrix entry: zero gradient
            assert abs(fd - g[key][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, idx)
