"""y = J x and z = M y in one call (r1s_matvec_prec, the operator of the
left-preconditioned system, section 6): parity with the CPU oracle (the
section 5.2 product, block-Jacobi by dense LU of the assembled diagonal
blocks) and with the two separate calls, on layouts the single kernel covers
(m <= 64, tridiagonal level band, no coupling, one right-hand side) and on
those that run the two kernels."""
import numpy as np
import pytest
import torch

from gpu_util import (DEV, U32, block_jacobi_ref, check_componentwise, host, log, matvec_scale,
                      sample_cells, to_dev, vec)
from oracle import ops
from paper_2403_09198_amd import gen, r1s
from paper_2403_09198_amd._lib import R1S_ERR_ARG, R1S_ERR_UNSUPPORTED

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
# the single kernel (float64: one pair per block; float32: every pair-count
# instantiation): small workload, degenerate meshes, m = 64 exactly, a
# ragged last workgroup (70 x 2 cells)
FUSED = [(16, 16, 8, (1, 1)), (1, 1, 1, (1, 1)), (5, 3, 2, (1, 1)), (7, 5, 61, (1, 1)),
         (70, 2, 6, (1, 1)), (7, 5, 61, (9, 2)), (5, 3, 20, (3, 0)), (4, 6, 61, (2, 6)),
         (3, 3, 8, (9, 6)), (2, 1, 1, (9, 6))]
# the two kernels: m > 64, wider level band, level/flow coupling
OTHER = [(3, 4, 62, (1, 1), 1, False), (2, 3, 125, (9, 2), 1, False), (7, 5, 61, (1, 1), 3, False),
         (7, 5, 61, (8, 6), 1, True), (5, 3, 8, (2, 1), 4, True)]


def _setup(nx, ny, L, ranks, band=1, arrow=False, seed=1):
    p = gen.make_problem(nx, ny, L, seed=seed, r_diag=ranks[0], r_off=ranks[1], band=band,
                         arrow=arrow)
    A = r1s.R1Matrix(nx, ny, L, to_dev(p), keep_f32=True, ranks=ranks, band=band, arrow=arrow)
    M = r1s.SMWPreconditioner(A, keep_f32=True)
    return p, A, M


def _per_cell_rel(z, ref):
    num = np.linalg.norm(z - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float(np.max(num / den))


def _check(p, nx, ny, L, A, M, x, ranks, band=1):
    m, P = L + 3, ranks[0] + 4 * ranks[1]
    xd = vec(x)
    yd, zd = M.apply_after_matvec(xd)
    y, z = host(yd), host(zd)
    ref = ops.matvec(p, nx, ny, L, x)
    sc = matvec_scale(p, nx, ny, L, x)
    check_componentwise(y, ref, sc, TOL64, "J x (fused call)")
    assert _per_cell_rel(z, block_jacobi_ref(p, nx, ny, L, ref)) <= TOL64
    # the two separate calls: the same J x, and M y to rounding
    y2 = A.matvec(xd)
    z2 = host(M.apply(y2))
    y2 = host(y2)
    ident = int(np.sum(y == y2)), int(np.sum(z == z2))
    log(f"  identical to the two calls: y {ident[0]}/{y.size}, z {ident[1]}/{z.size}")
    assert np.array_equal(y, y2)
    assert _per_cell_rel(z, z2) <= 1e-14
    # float32 values and factors: J x to the float32 matvec bound, and z to
    # the float32 apply bound measured against the oracle's M on that y
    y32, z32 = (host(t) for t in M.apply_after_matvec(xd, precision="f32"))
    check_componentwise(y32, ref, sc, (m + P + 2 * band + 16) * U32, "J x (fused, f32)")
    assert _per_cell_rel(z32, block_jacobi_ref(p, nx, ny, L, y32)) <= 8 * m * U32


@pytest.mark.parametrize("nx,ny,L,ranks", FUSED)
def test_fused_parity(nx, ny, L, ranks):
    log(f"fused matvec+apply nx={nx} ny={ny} L={L} ranks={ranks}")
    p, A, M = _setup(nx, ny, L, ranks)
    x = gen.make_vector(nx, ny, L, seed=4)
    _check(p, nx, ny, L, A, M, x, ranks)


@pytest.mark.parametrize("nx,ny,L,ranks,band,arrow", OTHER)
def test_two_kernel_layouts(nx, ny, L, ranks, band, arrow):
    log(f"matvec+apply (two kernels) nx={nx} ny={ny} L={L} ranks={ranks} band={band} arrow={arrow}")
    p, A, M = _setup(nx, ny, L, ranks, band, arrow)
    x = gen.make_vector(nx, ny, L, seed=5)
    _check(p, nx, ny, L, A, M, x, ranks, band)


def test_several_right_hand_sides():
    nx, ny, L = 9, 7, 61
    log(f"matvec+apply nrhs=3 nx={nx} ny={ny} L={L}")
    p, A, M = _setup(nx, ny, L, (1, 1))
    x = gen.make_vector(nx, ny, L, nrhs=3, seed=6)
    y, z = (host(t) for t in M.apply_after_matvec(vec(x)))
    ref = ops.matvec(p, nx, ny, L, x)
    check_componentwise(y, ref, matvec_scale(p, nx, ny, L, x), TOL64, "J x, 3 rhs")
    assert _per_cell_rel(z, block_jacobi_ref(p, nx, ny, L, ref)) <= TOL64


def test_full_size_sampled():
    # the 256 x 128, L = 61 workload, one pair per block, at full size
    nx, ny, L = 256, 128, 61
    log("fused matvec+apply full size 256x128 L=61")
    p, A, M = _setup(nx, ny, L, (1, 1), seed=0)
    x = gen.make_vector(nx, ny, L, seed=0)
    xd = vec(x)
    yd, zd = M.apply_after_matvec(xd)
    cells = sample_cells(nx, ny)
    y, z = host(yd)[:, cells], host(zd)[:, cells]
    ref = ops.matvec_rows(p, nx, ny, L, x, cells)
    check_componentwise(y, ref, matvec_scale(p, nx, ny, L, x, cells), TOL64, "J x sampled")
    rfull = np.zeros((1, nx * ny, L + 3))
    rfull[:, cells] = ref
    assert _per_cell_rel(z, block_jacobi_ref(p, nx, ny, L, rfull, cells)) <= TOL64
    y2 = A.matvec(xd)
    z2 = M.apply(y2)
    assert torch.equal(yd, y2)
    assert float(torch.max(torch.abs(zd - z2))) <= 1e-14 * float(torch.max(torch.abs(z2)))


def test_errors():
    nx, ny, L = 4, 3, 5
    p = gen.make_problem(nx, ny, L, seed=1)
    A = r1s.R1Matrix(nx, ny, L, to_dev(p))  # no float32 copy
    M = r1s.SMWPreconditioner(A)
    x = vec(gen.make_vector(nx, ny, L, seed=1))
    y, z = torch.empty_like(x), torch.empty_like(x)
    with pytest.raises(r1s.R1SError) as ei:
        M.apply_after_matvec(x, precision="f32")
    assert ei.value.code == R1S_ERR_ARG and "R1S_KEEP_F32" in str(ei.value)
    for yy, zz in ((x, z), (y, x), (y, y)):
        with pytest.raises(r1s.R1SError) as ei:
            r1s.r1s_matvec_prec(A.h, M.h, 0, 1, x, yy, zz)
        assert ei.value.code == R1S_ERR_ARG
    P = r1s.DenseLUPreconditioner(r1s.BSRMatrix(A))
    with pytest.raises(r1s.R1SError) as ei:
        r1s.r1s_matvec_prec(A.h, P.h, 0, 1, x, y, z)
    assert ei.value.code == R1S_ERR_UNSUPPORTED
    # a preconditioner of another matrix layout
    p2 = gen.make_problem(nx, ny, L, seed=2, r_diag=2)
    A2 = r1s.R1Matrix(nx, ny, L, to_dev(p2), ranks=(2, 1))
    M2 = r1s.SMWPreconditioner(A2)
    with pytest.raises(r1s.R1SError) as ei:
        r1s.r1s_matvec_prec(A.h, M2.h, 0, 1, x, y, z)
    assert ei.value.code == R1S_ERR_ARG
