"""Helpers shared by the GPU parity tests (marshalling and tolerances only)."""
import sys

import numpy as np
import torch

from oracle import assemble, blockjacobi, ops
from paper_2403_09198_amd import gen, r1s

DEV = "cuda:0"
U32 = 2.0 ** -24  # unit roundoff of float32


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(p):
    keys = gen.FIELDS + tuple(k for k in gen.PATTERN_FIELDS if k in p)
    return {k: torch.from_numpy(np.ascontiguousarray(p[k])).to(DEV) for k in keys}


def vec(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def abs_problem(p):
    return {k: np.abs(v) for k, v in p.items()}


def matvec_scale(p, nx, ny, L, x, cells=None, trans=False):
    """(|J| |x|) (or |J|^T |x|), the scale of a componentwise error bound."""
    pa = abs_problem(p)
    if cells is None:
        return (ops.matvec_T if trans else ops.matvec)(pa, nx, ny, L, np.abs(x))
    f = ops.matvec_T_rows if trans else ops.matvec_rows
    return f(pa, nx, ny, L, np.abs(x), cells)


def check_componentwise(y, ref, scale, tol, what):
    err = np.abs(y - ref)
    bad = err > tol * scale + 1e-300
    assert not bad.any(), (f"{what}: {int(bad.sum())} entries exceed {tol:g}*(|J||x|); "
                           f"worst ratio {np.max(err / (scale + 1e-300)):.3g}")


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def block_jacobi_ref(p, nx, ny, L, r, cells=None, trans=False):
    """Oracle z_c = D_cc^{-1} r_c (or D_cc^{-T}) by dense LU, for `cells`."""
    if cells is None:
        cells = list(range(nx * ny))
    D = assemble.diagonal_blocks(p, nx, ny, L, cells)
    LU, piv = blockjacobi.lu_factor(D)
    r3 = np.asarray(r)[:, cells, :] if np.ndim(r) == 3 else np.asarray(r)[None][:, cells, :]
    f = blockjacobi.lu_solve_T if trans else blockjacobi.lu_solve
    return np.stack([f(LU, piv, r3[i]) for i in range(r3.shape[0])])


def sample_cells(nx, ny, k=48, seed=0):
    rng = np.random.default_rng(seed)
    N = nx * ny
    fixed = {0, nx - 1, N - nx, N - 1, nx, nx + 1, N // 2}
    picks = set(rng.choice(N, size=min(k, N), replace=False).tolist())
    return sorted(c for c in fixed | picks if 0 <= c < N)
