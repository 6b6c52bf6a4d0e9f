"""The C ABI without Python in between: tests/abi_client.c (built by
__graft_entry__.build) reads a problem from a file, calls the library's
matvec, transposed matvec, SMW block-Jacobi apply (both directions), the
fused matvec + apply call and GMRES through include/r1s.h with its own hipMalloc'd buffers, and writes the
results; they are compared here with the CPU oracle (section 5.2, section 6
eq. SMW, right-preconditioned GMRES)."""
import os
import subprocess

import numpy as np
import pytest

from gpu_util import block_jacobi_ref, log, matvec_scale
from oracle import ops
from paper_2403_09198_amd import gen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CLIENT = os.path.join(HERE, "abi_client")
MAGIC = 0x31533152


def _write_problem(path, p, nx, ny, L, ranks, x, b):
    hdr = np.array([MAGIC, nx, ny, L, ranks[0], ranks[1]], dtype=np.int32)
    with open(path, "wb") as f:
        f.write(hdr.tobytes())
        for k in ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v"):
            f.write(np.ascontiguousarray(p[k], dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(x, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(b, dtype=np.float64).tobytes())


@pytest.mark.parametrize("nx,ny,L,ranks", [(7, 5, 8, (3, 1)), (4, 3, 61, (1, 1)),
                                           (3, 2, 125, (9, 2))])
def test_c_client_matches_oracle(tmp_path, nx, ny, L, ranks):
    if not os.path.exists(CLIENT):
        pytest.fail("tests/abi_client is not built (run __graft_entry__.build())")
    log(f"C client nx={nx} ny={ny} L={L} ranks={ranks}")
    p = gen.make_problem(nx, ny, L, seed=3, r_diag=ranks[0], r_off=ranks[1])
    x = gen.make_vector(nx, ny, L, seed=4)[0]
    b = gen.make_rhs(nx, ny, L, seed=5)[0]
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_problem(fin, p, nx, ny, L, ranks, x, b)
    r = subprocess.run([CLIENT, fin, fout], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    n = nx * ny * (L + 3)
    raw = open(fout, "rb").read()
    vals = np.frombuffer(raw[:7 * n * 8], dtype=np.float64).reshape(7, nx * ny, L + 3)
    iters, converged = np.frombuffer(raw[7 * n * 8:], dtype=np.int32)
    y, yt, z, zt, xs, yf, zf = vals
    sc, sct = matvec_scale(p, nx, ny, L, x[None])[0], matvec_scale(p, nx, ny, L, x[None], trans=True)[0]
    assert np.all(np.abs(y - ops.matvec(p, nx, ny, L, x)) <= 1e-12 * sc + 1e-300)
    assert np.all(np.abs(yt - ops.matvec_T(p, nx, ny, L, x)) <= 1e-12 * sct + 1e-300)
    for got, trans in ((z, False), (zt, True)):
        ref = block_jacobi_ref(p, nx, ny, L, x[None], trans=trans)[0]
        rel = np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)
        assert rel.max() <= 1e-12
    assert np.array_equal(yf, y)
    zref = block_jacobi_ref(p, nx, ny, L, y[None])[0]
    assert (np.linalg.norm(zf - zref, axis=-1) / np.linalg.norm(zref, axis=-1)).max() <= 1e-12
    assert converged == 1 and iters >= 1
    J = ops.dense_matrix(p, nx, ny, L)
    assert np.linalg.norm(b.ravel() - J @ xs.ravel()) <= 2e-12 * np.linalg.norm(b)
