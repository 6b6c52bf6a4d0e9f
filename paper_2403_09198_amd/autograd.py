"""Differentiable linear solve x = J^{-1} b through the r1s C ABI.

Forward: pack the structured values, set up the SMW block-Jacobi (with its
transposed factors) and solve by GMRES.  Only x is saved: backward solves
the adjoint system J^T lambda = dLoss/dx with a fresh Krylov basis (nothing
of the forward basis is stored), then forms the gradients w.r.t. b
(= lambda) and w.r.t. the structured arrays with the hand-written gradient
kernel.
"""
import torch

from . import r1s

FIELDS = r1s.FIELDS


class R1SolveFn(torch.autograd.Function):
    """apply(b, cfg, *arrays): arrays are the structured arrays the layout in
    cfg uses, in the order of r1s_inputs (FIELDS, then s_band and/or
    s_lev_flow, s_flow_lev)."""

    @staticmethod
    def forward(ctx, b, cfg, *arrays):
        nx, ny, L = cfg["nx"], cfg["ny"], cfg["L"]
        lay = r1s.layout(*cfg.get("ranks", (1, 1)), cfg.get("band", 1), cfg.get("arrow", False))
        names = r1s._used_fields(lay)
        vals = {k: t.detach().contiguous() for k, t in zip(names, arrays)}
        A = r1s.R1Matrix(nx, ny, L, vals, ranks=(lay.r_diag, lay.r_off), band=lay.band,
                         arrow=int(lay.arrow))
        M = r1s.SMWPreconditioner(A, with_trans=True)
        bb = b.detach().contiguous()
        res = r1s.gmres(A, M, bb, restart=cfg.get("restart", 50), rtol=cfg.get("rtol", 1e-12),
                        max_cycles=cfg.get("max_cycles", 200))
        ctx.A, ctx.M, ctx.cfg, ctx.names = A, M, cfg, names
        ctx.stats = res.stats
        ctx.save_for_backward(res.x)
        return res.x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        cfg = ctx.cfg
        gx = gx.contiguous()
        lam = r1s.gmres(ctx.A, ctx.M, gx, trans=True, restart=cfg.get("restart", 50),
                        rtol=cfg.get("adj_rtol", cfg.get("rtol", 1e-12)),
                        max_cycles=cfg.get("max_cycles", 200)).x
        g = r1s.grad(ctx.A, lam, x)
        return (lam, None) + tuple(g[k] for k in ctx.names)


def solve(b, values, nx, ny, L, **cfg):
    """x = J^{-1} b, differentiable w.r.t. b and every structured array.
    cfg: ranks=(r_diag, r_off) (default (1, 1)), band (default 1), arrow
    (default False), restart, rtol, adj_rtol, max_cycles."""
    c = dict(cfg, nx=nx, ny=ny, L=L)
    lay = r1s.layout(*c.get("ranks", (1, 1)), c.get("band", 1), c.get("arrow", False))
    return R1SolveFn.apply(b, c, *(values[k] for k in r1s._used_fields(lay)))
