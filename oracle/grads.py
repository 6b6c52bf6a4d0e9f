"""Gradients of the linear loss  Loss = sum_r w_r . x_r  with  J x_r = b_r.

Reverse-mode differentiation of a linear solve: with lambda_r = J^{-T} w_r,
dLoss/db_r = lambda_r and dLoss/dJ = -sum_r lambda_r x_r^T.  Restricting the
matrix cotangent to one dense block gives G_{c,d} = -sum_r lambda_r[c] x_r[nb]^T
(nb = the block's column cell); the chain rule through
D_{c,d} = S_{c,d} + u_{c,d} v_{c,d}^T then gives

    dS_{c,d}  = G_{c,d} at the stored pattern positions of S_{c,d}
    du_{c,d}  = G_{c,d} v_{c,d}
    dv_{c,d}  = G_{c,d}^T u_{c,d}

This works through the dense blocks (section 3's standard representation),
independent of any rank-one shortcut.
"""
import numpy as np

from . import assemble, mesh


def structured_grads(p, nx, ny, L, lam, x):
    """Gradients w.r.t. every stored structured array, summed over the batch.

    lam, x: [nrhs][N][m].  Returns a dict with the keys of the input arrays.
    """
    lam = np.asarray(lam, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    if lam.ndim == 2:
        lam, x = lam[None], x[None]
    N, m = nx * ny, L + 3
    band, arrow = mesh.pattern(p)
    ep = mesh.explicit_pattern(p)
    keys = ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v")
    if ep is not None:
        keys = ("s_cc", "s_nbr", "u", "v")
    elif (band, arrow) != (1, 0):
        keys = keys + ("s_band", "s_lev_flow", "s_flow_lev")
    g = {k: np.zeros_like(p[k]) for k in keys}
    for c in range(N):
        for d in (mesh.S, mesh.W, mesh.C, mesh.E, mesh.N):
            nb = mesh.neighbour(nx, ny, c, d)
            if nb < 0:
                continue
            G = -np.einsum("ri,rj->ij", lam[:, c, :], x[:, nb, :])
            a, cnt = mesh.pair_range(p, d)
            for q in range(a, a + cnt):
                g["u"][c, q] = G @ p["v"][c, q]
                g["v"][c, q] = G.T @ p["u"][c, q]
            if d == mesh.C and ep is not None:  # entry e of row i: G[i, indices[e]]
                pi, pj = ep
                for i in range(m):
                    for e in range(pi[i], pi[i + 1]):
                        g["s_cc"][c, e] = G[i, pj[e]]
            elif d == mesh.C:
                g["s_diag"][c] = np.diag(G)
                for k in range(L - 1):
                    g["s_sub"][c, k] = G[k + 1, k]
                    g["s_sup"][c, k] = G[k, k + 1]
                for t, (i, j) in enumerate(assemble.FLOW_PAIRS):
                    g["s_flow"][c, t] = G[L + i, L + j]
                for j in range(2, band + 1):
                    for k in range(j, L):
                        g["s_band"][c, j - 2, k] = G[k, k - j]
                    for k in range(0, L - j):
                        g["s_band"][c, band - 1 + j - 2, k] = G[k, k + j]
                if arrow:
                    for i in range(3):
                        g["s_lev_flow"][c, i] = G[:L, L + i]
                        g["s_flow_lev"][c, i] = G[L + i, :L]
                if arrow == 2:
                    g["s_lev_flow"][c, 3, :L - 1] = G[:L - 1, L - 1]
                    g["s_flow_lev"][c, 3, :L - 1] = G[L - 1, :L - 1]
            else:
                g["s_nbr"][c, mesh.NBR_SLOT[d]] = np.diag(G)
    return g


def loss(x, w):
    return float(np.sum(np.asarray(w) * np.asarray(x)))
