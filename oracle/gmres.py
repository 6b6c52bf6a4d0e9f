"""Restarted right-preconditioned GMRES (section 6; Saad & Schultz 1986).

Right preconditioning (eq. right_precond_system): solve (A M) y = b by GMRES
and return x = M y.  Because the preconditioner sits on the right, the
residual GMRES minimises is the true residual b - A x.

One cycle of GMRES(k): r0 = b - A x0, beta = |r0|, v_1 = r0 / beta; for
j = 1..k: w = A M v_j, modified Gram-Schmidt against v_1..v_j (giving the
Hessenberg column h_{1..j,j}), h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}.  Givens
rotations reduce H to upper-triangular form and carry beta e_1 along as g;
|g_{j+1}| is the residual norm of the current iterate.  At the end of the
cycle y solves R y = g and x = x0 + M V y.

Stopping: |b - A x| <= rtol |b|, checked on the true residual at the start of
every cycle.  A Hessenberg subdiagonal below 1e-14 |w before
orthogonalisation| ends the cycle early (the Krylov space is invariant).
"""
from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    converged: bool
    iters: int
    cycles: int
    rel_residual: float
    history: List[float] = field(default_factory=list)


def gmres(apply_A: Callable, apply_M: Callable, b, restart=30, rtol=1e-10,
          max_cycles=200, x0=None) -> GmresResult:
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    b = b.ravel()
    A = lambda v: np.ravel(apply_A(v.reshape(shape)))
    M = lambda v: np.ravel(apply_M(v.reshape(shape)))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64).ravel()
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return GmresResult(np.zeros(shape), True, 0, 0, 0.0)
    n = b.size
    iters = 0
    history = []
    for cycle in range(max_cycles + 1):
        r = b - A(x)
        beta = float(np.linalg.norm(r))
        history.append(beta / bnorm)
        if beta <= rtol * bnorm:
            return GmresResult(x.reshape(shape), True, iters, cycle, beta / bnorm, history)
        if cycle == max_cycles:
            break
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        jend = 0
        for j in range(restart):
            w = A(M(V[j]))
            w0 = float(np.linalg.norm(w))
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            iters += 1
            for i in range(j):  # previous rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = np.hypot(H[j, j], H[j + 1, j])
            breakdown = H[j + 1, j] <= 1e-14 * w0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            jend = j + 1
            if breakdown or abs(g[j + 1]) <= rtol * bnorm:
                break
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):  # back substitution R y = g
            y[i] = (g[i] - np.dot(H[i, i + 1:jend], y[i + 1:jend])) / H[i, i]
        x = x + M(V[:jend].T @ y)
    r = b - A(x)
    return GmresResult(x.reshape(shape), False, iters, max_cycles,
                       float(np.linalg.norm(r)) / bnorm, history)
