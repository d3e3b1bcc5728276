"""torch.autograd.Function around nys_pcg_solve / nys_pcg_backward.

x = (A + mu I)^{-1} b is differentiated with the adjoint (implicit-function)
formulas: lambda = (A + mu I)^{-1} dL/dx is solved with the same Nystrom
preconditioner, then dL/db = lambda, dL/dmu = -lambda^T x, and either
dL/dsigma = -lambda^T (dK/dsigma) x (RBF operator) or
dL/dX = -scale (X x lambda^T + X lambda x^T) (X^T X operator).
"""
from __future__ import annotations

import torch


class NystromSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, mu, sigma, data, kind, P, tol, maxit, prec, scale):
        from . import Operator, nys_pcg_solve
        op = Operator(kind, data.detach().contiguous(), data.shape[0] if kind == 2 else data.shape[1],
                      sigma=float(sigma), scale=float(scale))
        x, info = nys_pcg_solve(op, P, float(mu), b.detach(), tol=tol, maxit=maxit, prec=prec)
        ctx.save_for_backward(x, data)
        ctx.op, ctx.P, ctx.mu, ctx.tol, ctx.maxit, ctx.prec = op, P, float(mu), tol, maxit, prec
        ctx.kind = kind
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        from . import nys_pcg_backward
        x, data = ctx.saved_tensors
        want_sigma = ctx.kind == 2
        want_X = ctx.kind == 1 and ctx.needs_input_grad[3]
        r = nys_pcg_backward(ctx.op, ctx.P, ctx.mu, x, gx, want_sigma=want_sigma, want_X=want_X,
                             tol=ctx.tol, maxit=ctx.maxit, prec=ctx.prec)
        dev = x.device
        gmu = torch.tensor(r["gmu"], dtype=torch.float64, device=dev)
        gsig = torch.tensor(r["gsigma"], dtype=torch.float64, device=dev) if want_sigma else None
        gX = r["gX"].to(data.dtype) if want_X else None
        return r["gb"], gmu, gsig, gX, None, None, None, None, None, None


def nystrom_solve(b, mu, P, *, X=None, sigma=None, A=None, kind=None, tol=1e-10, maxit=500, prec=0,
                  scale=1.0):
    """Differentiable solve.  RBF: pass points X and bandwidth sigma (tensor or float);
    ridge: pass data X with kind=1 (A = scale X^T X); dense: pass A."""
    dev = b.device
    if A is not None:
        data, k = A, 0
    elif kind == 1:
        data, k = X, 1
    else:
        data, k = X, 2
    mu_t = mu if torch.is_tensor(mu) else torch.tensor(float(mu), dtype=torch.float64, device=dev)
    sig = sigma if sigma is not None else 0.0
    sig_t = sig if torch.is_tensor(sig) else torch.tensor(float(sig), dtype=torch.float64, device=dev)
    return NystromSolve.apply(b, mu_t, sig_t, data, k, P, tol, maxit, prec, scale)
