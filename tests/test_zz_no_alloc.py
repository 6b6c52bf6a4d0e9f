"""r1s_gmres_noalloc (the solve with the library's fixed workspace) against
r1s_gmres with a caller-owned workspace, through the C ABI: two calls in a
row on one GPU, the second with a smaller input, and the size limit."""
import numpy as np
import pytest
import torch

from gpu_util import host, log, relnorm, to_dev, vec
from paper_2403_09198_amd import _lib as L, gen, r1s

pytestmark = pytest.mark.gpu


def _pair(nx, ny, L_, nrhs, seed, **kw):
    p = gen.make_problem(nx, ny, L_, seed=seed)
    b = vec(gen.make_rhs(nx, ny, L_, nrhs=nrhs, seed=seed))
    A = r1s.R1Matrix(nx, ny, L_, to_dev(p), keep_f32=True)
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    ref = r1s.gmres(A, M, b, **kw)
    got = r1s.gmres(A, M, b, noalloc=True, **kw)
    return ref, got


@pytest.mark.parametrize("kw", [dict(restart=30, rtol=1e-10),
                                dict(restart=12, rtol=1e-11, mode="mixed"),
                                dict(restart=20, rtol=1e-10, trans=True, ortho="cgs2"),
                                dict(restart=20, rtol=1e-10, ortho="selective")])
def test_noalloc_matches_gmres_twice(kw):
    # first call: 16 x 16, L = 8, two right-hand sides; second: a smaller
    # input (5 x 4, L = 6, one right-hand side) through the same array
    for (nx, ny, L_, nrhs, seed) in ((16, 16, 8, 2, 3), (5, 4, 6, 1, 4)):
        log(f"noalloc vs gmres nx={nx} ny={ny} L={L_} nrhs={nrhs} {kw}")
        ref, got = _pair(nx, ny, L_, nrhs, seed, **kw)
        assert got.status == L.R1S_OK and ref.status == L.R1S_OK
        for r in range(nrhs):
            assert got.stats[r]["iters"] == ref.stats[r]["iters"]
            assert got.stats[r]["converged"] == 1
        # the same kernels in the same order: the same iterates
        assert relnorm(host(got.x), host(ref.x)) <= 1e-12


def test_noalloc_rejects_oversize():
    nx, ny, L_ = 128, 64, 61  # basis of 51 vectors of 4.2 MB: beyond 64 MiB
    p = gen.make_problem(nx, ny, L_, seed=0)
    A = r1s.R1Matrix(nx, ny, L_, to_dev(p))
    M = r1s.SMWPreconditioner(A)
    b = vec(gen.make_rhs(nx, ny, L_, seed=0))
    opts = L.GmresOpts(restart=50, max_cycles=200, rtol=1e-10)
    assert r1s.r1s_gmres_noalloc_size(A.h, opts, 1) > L.R1S_NOALLOC_MAX_BYTES
    with pytest.raises(r1s.R1SError) as ei:
        r1s.gmres(A, M, b, restart=50, noalloc=True)
    assert ei.value.code == L.R1S_ERR_ARG and "r1s_gmres_noalloc" in str(ei.value)
    # a smaller restart fits, and solves
    res = r1s.gmres(A, M, b, restart=4, max_cycles=500, noalloc=True)
    ref = r1s.gmres(A, M, b, restart=4, max_cycles=500)
    assert relnorm(host(res.x), host(ref.x)) <= 1e-12
