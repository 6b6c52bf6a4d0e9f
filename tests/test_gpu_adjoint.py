"""Adjoint / differentiation: R1SolveFn gradients against the oracle's
dense chain rule and central finite differences."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, host, log, relnorm, residual_bound, sample_cells, to_dev, vec
from oracle import grads as ograds, ops
from paper_2403_09198_amd import autograd, gen, r1s

pytestmark = pytest.mark.gpu
FIELDS = r1s.FIELDS


def _params(p):
    return {k: torch.from_numpy(p[k].copy()).to(DEV).requires_grad_(True) for k in FIELDS}


@pytest.mark.parametrize("nx,ny,L,nrhs", [(5, 4, 6, 3), (16, 16, 8, 2), (3, 2, 61, 1)])
def test_gradients_match_oracle(nx, ny, L, nrhs):
    log(f"adjoint oracle nx={nx} ny={ny} L={L} nrhs={nrhs}")
    p = gen.make_problem(nx, ny, L, seed=2)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=2)
    w = gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=2)
    params = _params(p)
    bt = vec(b).requires_grad_(True)
    x = autograd.solve(bt, params, nx, ny, L, rtol=1e-13)
    loss = (x * vec(w)).sum()
    loss.backward()
    # oracle: dense solves for x and lambda, chain rule through dense blocks
    J = ops.dense_matrix(p, nx, ny, L)
    n = nx * ny * (L + 3)
    X = np.linalg.solve(J, b.reshape(nrhs, n).T).T.reshape(b.shape)
    lam = np.linalg.solve(J.T, w.reshape(nrhs, n).T).T.reshape(b.shape)
    g = ograds.structured_grads(p, nx, ny, L, lam, X)
    assert relnorm(host(x), X) <= 1e-11
    assert relnorm(host(bt.grad), lam) <= 1e-10
    for k in FIELDS:
        assert relnorm(host(params[k].grad), g[k]) <= 1e-8, k


def test_gradients_finite_differences():
    nx, ny, L, nrhs = 4, 3, 5, 2
    log("adjoint finite differences")
    p = gen.make_problem(nx, ny, L, seed=3)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=3)
    w = vec(gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=3))
    params = _params(p)
    bt = vec(b).requires_grad_(True)
    (autograd.solve(bt, params, nx, ny, L, rtol=1e-14) * w).sum().backward()
    rng = np.random.default_rng(0)
    ex = gen.block_exists(nx, ny)
    h = 1e-6

    def loss_at(q):
        with torch.no_grad():
            vals = {k: vec(q[k]) for k in FIELDS}
            return float((autograd.solve(vec(b), vals, nx, ny, L, rtol=1e-14) * w).sum())

    for k in FIELDS:
        d = rng.standard_normal(p[k].shape)
        if k in ("u", "v"):
            d[~ex] = 0.0
        if k == "s_nbr":
            for j, dd in enumerate(gen.NBR_DIRS):
                d[~ex[:, dd], j] = 0.0
        qp = {kk: vv.copy() for kk, vv in p.items()}
        qm = {kk: vv.copy() for kk, vv in p.items()}
        qp[k] = p[k] + h * d
        qm[k] = p[k] - h * d
        fd = (loss_at(qp) - loss_at(qm)) / (2 * h)
        an = float(np.sum(host(params[k].grad) * d))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, fd, an)


def test_adjoint_batch_full_size_properties():
    # the 256 x 128, L = 61 batch-of-8 adjoint workload: lambda = dL/db solves
    # J^T lambda = w and x solves J x = b, both checked by the oracle's rows
    # (transposed / forward) on the sampled cells of the forward parity
    # checks; the structured gradients agree with the oracle's dense chain
    # rule on the same cells
    nx, ny, L, nrhs = 256, 128, 61, 8
    log("adjoint full size batch 8")
    p = gen.make_problem(nx, ny, L, seed=0)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=0)
    w = gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=0)
    params = _params(p)
    bt = vec(b).requires_grad_(True)
    rtol = 1e-12
    x = autograd.solve(bt, params, nx, ny, L, rtol=rtol)
    (x * vec(w)).sum().backward()
    lam = host(bt.grad)
    X = host(x)
    cells = sample_cells(nx, ny)
    K = 5 * (L + 3) + 17  # terms of a row: the oracle's dense block rows
    rr = w[:, cells] - ops.matvec_T_rows(p, nx, ny, L, lam, cells)
    bound = residual_bound(p, nx, ny, L, w, lam, rtol, K, cells, trans=True)
    for r in range(nrhs):
        assert np.linalg.norm(rr[r]) <= bound[r], (r, np.linalg.norm(rr[r]), bound[r])
    rx = b[:, cells] - ops.matvec_rows(p, nx, ny, L, X, cells)
    bound = residual_bound(p, nx, ny, L, b, X, rtol, K, cells)
    for r in range(nrhs):
        assert np.linalg.norm(rx[r]) <= bound[r], (r, np.linalg.norm(rx[r]), bound[r])
    # the oracle's dense-block chain rule at full size, compared on sampled cells
    g = ograds.structured_grads(p, nx, ny, L, lam, X)
    for k in FIELDS:
        gk = host(params[k].grad)
        assert relnorm(gk[cells], g[k][cells]) <= 1e-8, k
    assert relnorm(host(params["u"].grad), g["u"]) <= 1e-8


def test_full_size_finite_differences():
    # central differences of the batch-of-8 loss sum(w . x) at 256 x 128,
    # L = 61, along two random directions per parameter array (b and each
    # structured array), each supported on 16 random cells, against the
    # directional derivative of the R1SolveFn gradients.
    #
    # The quotient is formed as sum(w . (x(+h) - x(-h))) / 2h: differencing
    # the solutions before the sum keeps the float64 rounding of the
    # 16.7-million-term loss out of it.  Error budget: the truncation error
    # (h^2 / 6 = 1.7e-13 times the third derivative of the loss along d) and
    # the solve noise (|e+| + |e-|) / 2h, e+- the errors of w . x(+-h) for
    # solves to rtol = 1e-14.  Their size is measured as
    # e_x = |w . (x_a - x_b)| for two solves of the unperturbed system to the
    # same tolerance from different starting points (zero, and a random
    # vector of norm 1e-6 |x|); the quotient must agree with the gradient to
    # 1e-5 of sum |g_i d_i| plus 2 e_x / h.
    nx, ny, L, nrhs = 256, 128, 61, 8
    log("adjoint full-size finite differences")
    p = gen.make_problem(nx, ny, L, seed=0)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=0)
    wd = vec(gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=0))
    params = _params(p)
    bt = vec(b).requires_grad_(True)
    (autograd.solve(bt, params, nx, ny, L, rtol=1e-14, adj_rtol=1e-14) * wd).sum().backward()
    grads = {k: params[k].grad.detach() for k in FIELDS}
    grads["b"] = bt.grad.detach()
    base = {k: params[k].detach() for k in FIELDS}
    bd = vec(b)

    def x_at(vals, bb, x0=None):
        A = r1s.R1Matrix(nx, ny, L, vals)
        M = r1s.SMWPreconditioner(A)
        return r1s.gmres(A, M, bb, x0=x0, restart=50, rtol=1e-14).x

    def wdot(dx):
        return float(torch.sum(wd * dx, dtype=torch.float64))

    xa = x_at(base, bd)
    x0 = torch.randn_like(xa)
    x0 *= 1e-6 * float(torch.linalg.norm(xa)) / float(torch.linalg.norm(x0))
    e_x = abs(wdot(xa - x_at(base, bd, x0=xa + x0)))
    h = 1e-6
    rng = np.random.default_rng(7)
    ex = gen.block_exists(nx, ny)
    N = nx * ny
    for k in list(FIELDS) + ["b"]:
        shape = tuple(grads[k].shape)
        for trial in range(2):
            cells = rng.choice(N, size=16, replace=False)
            d = np.zeros(shape)
            if k == "b":
                d[:, cells] = rng.standard_normal((nrhs, 16) + shape[2:])
            else:
                d[cells] = rng.standard_normal((16,) + shape[1:])
            if k in ("u", "v"):
                d[~ex] = 0.0
            if k == "s_nbr":
                for j, dd in enumerate(gen.NBR_DIRS):
                    d[~ex[:, dd], j] = 0.0
            d /= np.linalg.norm(d)
            dt = vec(d)
            if k == "b":
                xp, xm = x_at(base, bd + h * dt), x_at(base, bd - h * dt)
            else:
                xp = x_at(dict(base, **{k: base[k] + h * dt}), bd)
                xm = x_at(dict(base, **{k: base[k] - h * dt}), bd)
            fd = wdot(xp - xm) / (2 * h)
            gk = grads[k]
            an = float(torch.sum(gk * dt))
            scale = float(torch.sum(torch.abs(gk) * torch.abs(dt)))
            tol = 1e-5 * scale + 2 * e_x / h
            log(f"  {k} #{trial}: fd {fd:.10g} grad {an:.10g} diff {abs(fd - an):.3g} "
                f"scale {scale:.3g} noise {2 * e_x / h:.3g} tol {tol:.3g}")
            assert abs(fd - an) <= tol, (k, trial, fd, an, tol)
