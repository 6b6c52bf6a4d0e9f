"""Adjoint / differentiation: R1SolveFn gradients against the oracle's
dense chain rule and central finite differences."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, host, log, relnorm, to_dev, vec
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
    # the 256 x 128, L = 61 batch-of-8 adjoint workload: gradients w.r.t. b
    # solve J^T lambda = w (checked by the oracle's transposed rows), and the
    # structured gradients agree with the oracle's dense chain rule on
    # sampled cells
    nx, ny, L, nrhs = 256, 128, 61, 8
    log("adjoint full size batch 8")
    p = gen.make_problem(nx, ny, L, seed=0)
    b = gen.make_rhs(nx, ny, L, nrhs=nrhs, seed=0)
    w = gen.make_loss_weights(nx, ny, L, nrhs=nrhs, seed=0)
    params = _params(p)
    bt = vec(b).requires_grad_(True)
    x = autograd.solve(bt, params, nx, ny, L, rtol=1e-12)
    (x * vec(w)).sum().backward()
    lam = host(bt.grad)
    X = host(x)
    cells = [0, 255, 256 * 64 + 17, 256 * 127, 256 * 128 - 1]
    rr = w[:, cells] - ops.matvec_T_rows(p, nx, ny, L, lam, cells)
    assert np.max(np.abs(rr)) <= 1e-10 * np.max(np.abs(w))
    # the oracle's dense-block chain rule at full size, compared on sampled cells
    g = ograds.structured_grads(p, nx, ny, L, lam, X)
    for k in FIELDS:
        gk = host(params[k].grad)
        assert relnorm(gk[cells], g[k][cells]) <= 1e-8, k
    assert relnorm(host(params["u"].grad), g["u"]) <= 1e-8
