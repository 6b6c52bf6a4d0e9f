"""C ABI behaviour on the GPU: value updates, flag errors, random shapes."""
import numpy as np
import pytest
import torch

from gpu_util import (DEV, U32, block_jacobi_ref, check_componentwise, host, log, matvec_scale,
                      relnorm, to_dev, vec)
from oracle import ops
from paper_2403_09198_amd import gen, r1s
from paper_2403_09198_amd._lib import R1S_ERR_ARG, R1S_ERR_UNSUPPORTED

pytestmark = pytest.mark.gpu


def test_update_values_same_structure():
    nx, ny, L = 9, 6, 13
    p1 = gen.make_problem(nx, ny, L, seed=1)
    p2 = gen.make_problem(nx, ny, L, seed=2)
    A = r1s.R1Matrix(nx, ny, L, to_dev(p1), keep_f32=True)
    x = gen.make_vector(nx, ny, L, nrhs=2, seed=3)
    A.update(to_dev(p2))
    y = host(A.matvec(vec(x)))
    check_componentwise(y, ops.matvec(p2, nx, ny, L, x), matvec_scale(p2, nx, ny, L, x), 1e-12,
                        "J x after update")
    y32 = host(A.matvec(vec(x), precision="f32"))
    check_componentwise(y32, ops.matvec(p2, nx, ny, L, x), matvec_scale(p2, nx, ny, L, x),
                        (L + 3 + 16) * U32, "f32 J x after update")
    M = r1s.SMWPreconditioner(A)
    z = host(M.apply(vec(x)))
    ref = block_jacobi_ref(p2, nx, ny, L, x)
    assert relnorm(z, ref) <= 1e-12


def test_flag_errors():
    nx, ny, L = 4, 3, 5
    p = gen.make_problem(nx, ny, L, seed=1)
    A = r1s.R1Matrix(nx, ny, L, to_dev(p))  # no float32 copy
    M = r1s.SMWPreconditioner(A)              # no transposed factors
    x = vec(gen.make_vector(nx, ny, L, seed=1))
    with pytest.raises(r1s.R1SError) as ei:
        A.matvec(x, precision="f32")
    assert ei.value.code == R1S_ERR_ARG and "R1S_KEEP_F32" in str(ei.value)
    with pytest.raises(r1s.R1SError) as ei:
        M.apply(x, trans=True)
    assert ei.value.code == R1S_ERR_ARG and "R1S_WITH_TRANS" in str(ei.value)
    with pytest.raises(r1s.R1SError) as ei:
        M.apply(x, precision="f32")
    assert ei.value.code == R1S_ERR_ARG
    with pytest.raises(r1s.R1SError) as ei:
        r1s.gmres(A, M, x, trans=True)
    assert ei.value.code == R1S_ERR_ARG
    with pytest.raises(r1s.R1SError) as ei:
        r1s.gmres(A, M, x, mode="mixed")
    assert ei.value.code == R1S_ERR_ARG
    B = r1s.BSRMatrix(A)
    P = r1s.DenseLUPreconditioner(B)
    with pytest.raises(r1s.R1SError) as ei:
        r1s.r1s_prec_apply(P.h, 0, 1, 1, x, torch.empty_like(x))
    assert ei.value.code == R1S_ERR_UNSUPPORTED
    with pytest.raises(r1s.R1SError) as ei:
        A.matvec(x, out=x)
    assert ei.value.code == R1S_ERR_ARG


def test_wrong_sizes_are_rejected_by_the_binding():
    nx, ny, L = 4, 3, 5
    p = gen.make_problem(nx, ny, L, seed=1)
    vals = to_dev(p)
    bad = dict(vals)
    bad["u"] = vals["u"][:, :4].contiguous()
    with pytest.raises(ValueError):
        r1s.R1Matrix(nx, ny, L, bad)
    A = r1s.R1Matrix(nx, ny, L, vals)
    with pytest.raises(ValueError):
        A.matvec(torch.zeros(7, dtype=torch.float64, device=DEV))
    with pytest.raises(TypeError):
        A.matvec(torch.zeros(nx * ny * (L + 3), dtype=torch.float32, device=DEV))


RNG = np.random.default_rng(2026)
RANDOM_SHAPES = [(int(RNG.integers(1, 9)), int(RNG.integers(1, 9)), int(RNG.integers(1, 254)),
                  int(RNG.integers(1, 5))) for _ in range(12)]


@pytest.mark.parametrize("nx,ny,L,nrhs", RANDOM_SHAPES)
def test_random_shapes(nx, ny, L, nrhs):
    log(f"random shape nx={nx} ny={ny} L={L} nrhs={nrhs}")
    p = gen.make_problem(nx, ny, L, seed=nx * 1000 + ny * 100 + L)
    A = r1s.R1Matrix(nx, ny, L, to_dev(p), keep_f32=True)
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    x = gen.make_vector(nx, ny, L, nrhs=nrhs, seed=L)
    xd = vec(x)
    for trans in (False, True):
        ref = (ops.matvec_T if trans else ops.matvec)(p, nx, ny, L, x)
        sc = matvec_scale(p, nx, ny, L, x, trans=trans)
        check_componentwise(host(A.matvec(xd, trans=trans)), ref, sc, 1e-12, "J x")
        check_componentwise(host(A.matvec(xd, trans=trans, precision="f32")), ref, sc,
                            (L + 3 + 16) * U32, "J x f32")
        z = host(M.apply(xd, trans=trans))
        zr = block_jacobi_ref(p, nx, ny, L, x, trans=trans)
        num = np.linalg.norm(z - zr, axis=-1)
        den = np.maximum(np.linalg.norm(zr, axis=-1), 1e-300)
        assert float(np.max(num / den)) <= 1e-12
