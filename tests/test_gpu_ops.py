"""GPU parity of the operator kernels (matvec, transpose, SMW apply, BSR)
against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from gpu_util import (DEV, U32, block_jacobi_ref, check_componentwise, host, log, matvec_scale,
                      relnorm, sample_cells, to_dev, vec)
from oracle import ops, storage
from paper_2403_09198_amd import gen, r1s

pytestmark = pytest.mark.gpu

# (nx, ny, L): the small workload, degenerate meshes, and block sizes on both
# sides of every 64-lane boundary up to m = 256
SHAPES = [(16, 16, 8), (1, 1, 1), (3, 2, 1), (1, 5, 2), (5, 3, 2), (7, 5, 61), (3, 4, 62),
          (2, 3, 125), (2, 2, 126), (3, 2, 200), (2, 3, 253)]
TOL64 = 1e-12


def _setup(nx, ny, L, seed=1, keep_f32=True, with_trans=True):
    p = gen.make_problem(nx, ny, L, seed=seed)
    A = r1s.R1Matrix(nx, ny, L, to_dev(p), keep_f32=keep_f32)
    M = r1s.SMWPreconditioner(A, keep_f32=keep_f32, with_trans=with_trans)
    return p, A, M


@pytest.mark.parametrize("nx,ny,L", SHAPES)
@pytest.mark.parametrize("nrhs", [1, 3, 11])  # 11 = batches of 8, 2 and 1
def test_matvec_parity(nx, ny, L, nrhs):
    log(f"matvec parity nx={nx} ny={ny} L={L} nrhs={nrhs}")
    p, A, M = _setup(nx, ny, L)
    x = gen.make_vector(nx, ny, L, nrhs=nrhs, seed=4)
    xd = vec(x)
    y = host(A.matvec(xd))
    ref = ops.matvec(p, nx, ny, L, x)
    assert relnorm(y, ref) <= TOL64
    check_componentwise(y, ref, matvec_scale(p, nx, ny, L, x), TOL64, "J x")
    yt = host(A.matvec(xd, trans=True))
    reft = ops.matvec_T(p, nx, ny, L, x)
    assert relnorm(yt, reft) <= TOL64
    check_componentwise(yt, reft, matvec_scale(p, nx, ny, L, x, trans=True), TOL64, "J^T x")
    # float32 values, float32 accumulation: each entry is a sum of at most
    # m + 12 rounded products of rounded operands
    tol32 = (nx * 0 + L + 3 + 16) * U32
    y32 = host(A.matvec(xd, precision="f32"))
    check_componentwise(y32, ref, matvec_scale(p, nx, ny, L, x), tol32, "J x (f32)")
    yt32 = host(A.matvec(xd, trans=True, precision="f32"))
    check_componentwise(yt32, reft, matvec_scale(p, nx, ny, L, x, trans=True), tol32, "J^T x (f32)")
    # residual r = b - J x in float64
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=4)
    r = host(A.residual(vec(b), xd))
    check_componentwise(r, b - ref, matvec_scale(p, nx, ny, L, x) + np.abs(b), TOL64, "b - J x")


def _per_cell_rel(z, ref):
    num = np.linalg.norm(z - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float(np.max(num / den))


@pytest.mark.parametrize("nx,ny,L", SHAPES)
@pytest.mark.parametrize("nrhs", [1, 5, 13])  # 13 = batches of 8, 4 and 1
def test_smw_apply_parity(nx, ny, L, nrhs):
    log(f"smw apply parity nx={nx} ny={ny} L={L} nrhs={nrhs}")
    p, A, M = _setup(nx, ny, L)
    r = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=6)
    rd = vec(r)
    ref = block_jacobi_ref(p, nx, ny, L, r)
    z = host(M.apply(rd))
    assert _per_cell_rel(z, ref) <= TOL64
    reft = block_jacobi_ref(p, nx, ny, L, r, trans=True)
    zt = host(M.apply(rd, trans=True))
    assert _per_cell_rel(zt, reft) <= TOL64
    # float32 factors and arithmetic: blocks are diagonally dominant with
    # small condition numbers, so the error is a few m * u32 relative
    tol32 = 8 * (L + 3) * U32
    assert _per_cell_rel(host(M.apply(rd, precision="f32")), ref) <= tol32
    assert _per_cell_rel(host(M.apply(rd, trans=True, precision="f32")), reft) <= tol32


def test_full_size_sampled_parity():
    # the 256 x 128, L = 61 workload at full size, checked on sampled cells
    nx, ny, L = 256, 128, 61
    log("full-size sampled parity 256x128 L=61")
    p, A, M = _setup(nx, ny, L, seed=0)
    x = gen.make_vector(nx, ny, L, seed=0)
    xd = vec(x)
    cells = sample_cells(nx, ny)
    y = host(A.matvec(xd))[:, cells]
    ref = ops.matvec_rows(p, nx, ny, L, x, cells)
    check_componentwise(y, ref, matvec_scale(p, nx, ny, L, x, cells), TOL64, "J x sampled")
    yt = host(A.matvec(xd, trans=True))[:, cells]
    reft = ops.matvec_T_rows(p, nx, ny, L, x, cells)
    check_componentwise(yt, reft, matvec_scale(p, nx, ny, L, x, cells, trans=True), TOL64,
                        "J^T x sampled")
    z = host(M.apply(xd))[:, cells]
    assert _per_cell_rel(z, block_jacobi_ref(p, nx, ny, L, x, cells)) <= TOL64
    zt = host(M.apply(xd, trans=True))[:, cells]
    assert _per_cell_rel(zt, block_jacobi_ref(p, nx, ny, L, x, cells, trans=True)) <= TOL64
    # adjoint identity <w, J x> = <J^T w, x> over the whole mesh
    w = gen.make_vector(nx, ny, L, seed=1)
    wd = vec(w)
    lhs = float(torch.dot(wd.ravel(), A.matvec(xd).ravel()))
    rhs = float(torch.dot(A.matvec(wd, trans=True).ravel(), xd.ravel()))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + float(torch.linalg.norm(wd)) * float(torch.linalg.norm(xd)))


@pytest.mark.parametrize("L", [32, 120, 200])
def test_level_sweep_full_size_sampled_parity(L):
    # the 512 x 256 level-sweep workloads at full size (m = 35 / 123 / 203:
    # one wave per cell, and workgroups of 2 and 4 waves), sampled cells
    nx, ny = 512, 256
    log(f"level sweep full-size sampled parity 512x256 L={L}")
    p, A, M = _setup(nx, ny, L, seed=0, keep_f32=False)
    x = gen.make_vector(nx, ny, L, seed=0)
    xd = vec(x)
    cells = sample_cells(nx, ny, k=32, seed=L)
    y = host(A.matvec(xd))[:, cells]
    check_componentwise(y, ops.matvec_rows(p, nx, ny, L, x, cells),
                        matvec_scale(p, nx, ny, L, x, cells), TOL64, "J x sampled")
    yt = host(A.matvec(xd, trans=True))[:, cells]
    check_componentwise(yt, ops.matvec_T_rows(p, nx, ny, L, x, cells),
                        matvec_scale(p, nx, ny, L, x, cells, trans=True), TOL64, "J^T x sampled")
    z = host(M.apply(xd))[:, cells]
    assert _per_cell_rel(z, block_jacobi_ref(p, nx, ny, L, x, cells)) <= TOL64
    zt = host(M.apply(xd, trans=True))[:, cells]
    assert _per_cell_rel(zt, block_jacobi_ref(p, nx, ny, L, x, cells, trans=True)) <= TOL64
    del A, M
    torch.cuda.empty_cache()


def test_bitwise_deterministic():
    p, A, M = _setup(64, 32, 61, seed=3)
    x = vec(gen.make_vector(64, 32, 61, nrhs=2, seed=2))
    for f in (lambda: A.matvec(x), lambda: A.matvec(x, trans=True), lambda: M.apply(x),
              lambda: M.apply(x, trans=True)):
        a, b = f(), f()
        assert torch.equal(a, b)


@pytest.mark.parametrize("L", [8, 61])
def test_batched_apply_equals_one_at_a_time(L):
    # several right-hand sides per launch share the coefficient half of the
    # sweeps' scans; the results agree with one right-hand side per launch
    # to rounding (8 = one launch of eight, 7 = 4 + 2 + 1)
    nx, ny = 9, 7
    log(f"batched apply vs single nx={nx} ny={ny} L={L}")
    p, A, M = _setup(nx, ny, L, seed=5)
    for nrhs in (8, 7):
        r = vec(gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=nrhs))
        for trans in (False, True):
            for prec, tol in (("f64", 1e-14), ("f32", 8 * (L + 3) * U32)):
                zb = host(M.apply(r, trans=trans, precision=prec))
                zs = np.concatenate([host(M.apply(r[i:i + 1].contiguous(), trans=trans,
                                                  precision=prec)) for i in range(nrhs)])
                log(f"  nrhs={nrhs} trans={trans} {prec}: {int(np.sum(zb == zs))}/{zb.size} equal")
                assert _per_cell_rel(zb, zs) <= tol, (nrhs, trans, prec)


@pytest.mark.parametrize("nx,ny,L", [(16, 16, 8), (1, 1, 1), (5, 3, 2), (7, 5, 61), (3, 4, 62),
                                     (2, 3, 125), (3, 2, 200)])
def test_bsr_parity(nx, ny, L):
    log(f"bsr parity nx={nx} ny={ny} L={L}")
    p, A, M = _setup(nx, ny, L, keep_f32=False, with_trans=False)
    B = r1s.BSRMatrix(A)
    P = r1s.DenseLUPreconditioner(B)
    x = gen.make_vector(nx, ny, L, nrhs=2, seed=9)
    xd = vec(x)
    ref = ops.matvec(p, nx, ny, L, x)
    y = host(B.matvec(xd))
    check_componentwise(y, ref, matvec_scale(p, nx, ny, L, x), TOL64, "BSR J x")
    z = host(P.apply(xd))
    assert _per_cell_rel(z, block_jacobi_ref(p, nx, ny, L, x)) <= TOL64


def test_storage_counts():
    for nx, ny, L in [(16, 16, 8), (256, 128, 61), (3, 1, 4)]:
        p = gen.make_problem(nx, ny, L, seed=0) if nx * ny * (L + 3) < 10 ** 6 else None
        if p is None:
            p = {k: np.zeros(s) for k, s in [
                ("s_diag", (nx * ny, L + 3)), ("s_sub", (nx * ny, L - 1)),
                ("s_sup", (nx * ny, L - 1)), ("s_flow", (nx * ny, 6)),
                ("s_nbr", (nx * ny, 4, L + 3)), ("u", (nx * ny, 5, L + 3)),
                ("v", (nx * ny, 5, L + 3))]}
        A = r1s.R1Matrix(nx, ny, L, to_dev(p))
        s = A.storage()
        m = L + 3
        assert s["structured_values"] == storage.structured_values(nx, ny, m)
        assert s["bsr_values"] == storage.bsr_values(nx, ny, m)
        assert s["n_blocks"] == storage.n_blocks(nx, ny)


# Meshes whose rows span several packed tiles: one pair per block, m not a
# multiple of 64 (Q = floor(1024 / m) cells per workgroup; the matvec tiles
# are Q cells of a row inside one of eight column bands, the last ragged),
# nx below, at and above the band count.
PACKED_SHAPES = [(50, 3, 200), (61, 3, 126), (250, 2, 32), (37, 5, 32), (9, 4, 62), (5, 7, 120),
                 (17, 3, 29), (3, 11, 70)]


@pytest.mark.parametrize("nx,ny,L", PACKED_SHAPES)
def test_packed_parity(nx, ny, L):
    log(f"packed parity nx={nx} ny={ny} L={L}")
    p, A, M = _setup(nx, ny, L, seed=2)
    x = gen.make_vector(nx, ny, L, seed=8)
    xd = vec(x)
    ref = ops.matvec(p, nx, ny, L, x)
    sc = matvec_scale(p, nx, ny, L, x)
    check_componentwise(host(A.matvec(xd)), ref, sc, TOL64, "J x")
    reft = ops.matvec_T(p, nx, ny, L, x)
    sct = matvec_scale(p, nx, ny, L, x, trans=True)
    check_componentwise(host(A.matvec(xd, trans=True)), reft, sct, TOL64, "J^T x")
    tol32 = (L + 3 + 16) * U32
    check_componentwise(host(A.matvec(xd, precision="f32")), ref, sc, tol32, "J x (f32)")
    check_componentwise(host(A.matvec(xd, trans=True, precision="f32")), reft, sct, tol32,
                        "J^T x (f32)")
    b = gen.make_rhs(nx, ny, L, seed=3)
    check_componentwise(host(A.residual(vec(b), xd)), b - ref, sc + np.abs(b), TOL64, "b - J x")
    zr = block_jacobi_ref(p, nx, ny, L, x)
    assert _per_cell_rel(host(M.apply(xd)), zr) <= TOL64
    zrt = block_jacobi_ref(p, nx, ny, L, x, trans=True)
    assert _per_cell_rel(host(M.apply(xd, trans=True)), zrt) <= TOL64
    tol32a = 8 * (L + 3) * U32
    assert _per_cell_rel(host(M.apply(xd, precision="f32")), zr) <= tol32a
    assert _per_cell_rel(host(M.apply(xd, trans=True, precision="f32")), zrt) <= tol32a
    # every output entry written: poisoned outputs must be overwritten
    y = torch.full_like(xd, float("nan"))
    A.matvec(xd, out=y)
    z = torch.full_like(xd, float("nan"))
    M.apply(xd, out=z)
    assert bool(torch.isfinite(y).all()) and bool(torch.isfinite(z).all())
