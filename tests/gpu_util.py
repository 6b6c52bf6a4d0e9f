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


U64 = 2.0 ** -53  # unit roundoff of float64


def gamma(k, u=U64):
    """gamma_k = k u / (1 - k u): the bound on the relative rounding error of
    a sum of k products (Higham, Accuracy and Stability, Lemma 3.1)."""
    return k * u / (1.0 - k * u)


def residual_bound(p, nx, ny, L, b, x, rtol, terms, cells=None, trans=False):
    """What the oracle's residual b - J x may reach, in the 2-norm over the
    block rows `cells` (all by default), for an x whose float64 residual the
    library computed to be at most rtol |b|_2 per right-hand side: the
    library's residual on those rows (at most its whole norm) plus the
    difference of two float64 evaluations of b - J x, each within
    gamma_terms (|J||x| + |b|) componentwise.  Returns one bound per
    right-hand side."""
    b3 = np.asarray(b)
    x3 = np.asarray(x)
    scale = matvec_scale(p, nx, ny, L, x3, cells, trans)
    bc = b3 if cells is None else b3[:, cells]
    s = scale + np.abs(bc)
    nb = np.linalg.norm(b3.reshape(b3.shape[0], -1), axis=1)
    ns = np.linalg.norm(s.reshape(s.shape[0], -1), axis=1)
    return rtol * nb + 2.0 * gamma(terms) * ns
