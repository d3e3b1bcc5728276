"""torch.autograd.Functions around the solve and the RBF cross products.

NystromSolve: x = (A + mu I)^{-1} b, differentiated with the adjoint
(implicit-function) formulas: lambda = (A + mu I)^{-1} dL/dx is solved with the
same Nystrom preconditioner (A is symmetric), then dL/db = lambda,
dL/dmu = -lambda^T x, and either dL/dsigma = -lambda^T (dK/dsigma) x (RBF
operator) or dL/dX = -scale (X x lambda^T + X lambda x^T) (X^T X operator).
The preconditioner is not differentiated: for any symmetric positive definite
P, PCG converges to the same x, so x does not depend on P.

RbfCross: u = K(Xv, X; sigma) v for held-out points Xv (a validation loss),
with dL/dv = K^T g and dL/dsigma = g^T (dK/dsigma) v.

Gradients the library does not form (dense A data, RBF point coordinates)
raise instead of being returned as zero, and a forward or adjoint solve that
does not reach its tolerance raises NysError.
"""
from __future__ import annotations

import torch

OP_DENSE, OP_XTX, OP_RBF = 0, 1, 2


class NystromSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, mu, sigma, data, kind, P, tol, maxit, prec, scale, inner_tol):
        from . import Operator, nys_pcg_solve
        n = data.shape[0] if kind == OP_RBF else data.shape[1]
        op = Operator(kind, data.detach().contiguous(), n, sigma=float(sigma), scale=float(scale))
        x, info = nys_pcg_solve(op, P, float(mu), b.detach(), tol=tol, maxit=maxit, prec=prec,
                                inner_tol=inner_tol, raise_on_not_converged=True)
        ctx.save_for_backward(x, data)
        ctx.op, ctx.P, ctx.mu, ctx.tol, ctx.maxit, ctx.prec = op, P, float(mu), tol, maxit, prec
        ctx.inner_tol = inner_tol
        ctx.kind = kind
        ctx.info = info
        ctx.mu_shape, ctx.sigma_shape = mu.shape, sigma.shape
        return x

    @staticmethod
    def backward(ctx, gx):
        from . import nys_pcg_backward
        x, data = ctx.saved_tensors
        if ctx.needs_input_grad[3] and ctx.kind != OP_XTX:
            raise NotImplementedError(
                "nystrom_solve: the gradient with respect to %s is not formed; detach it"
                % ("the dense matrix A" if ctx.kind == OP_DENSE else "the RBF points X"))
        want_sigma = ctx.kind == OP_RBF and ctx.needs_input_grad[2]
        want_X = ctx.kind == OP_XTX and ctx.needs_input_grad[3]
        r = nys_pcg_backward(ctx.op, ctx.P, ctx.mu, x, gx, want_sigma=want_sigma, want_X=want_X,
                             tol=ctx.tol, maxit=ctx.maxit, prec=ctx.prec, inner_tol=ctx.inner_tol,
                             raise_on_not_converged=True)
        dev = x.device
        # scalar gradients in the shape of the inputs they belong to
        gmu = (torch.tensor(r["gmu"], dtype=torch.float64, device=dev).reshape(ctx.mu_shape)
               if ctx.needs_input_grad[1] else None)
        gsig = (torch.tensor(r["gsigma"], dtype=torch.float64, device=dev).reshape(ctx.sigma_shape)
                if want_sigma else None)
        gX = r["gX"].to(data.dtype) if want_X else None
        gb = r["gb"] if ctx.needs_input_grad[0] else None
        return gb, gmu, gsig, gX, None, None, None, None, None, None, None


def nystrom_solve(b, mu, P, *, X=None, sigma=None, A=None, kind=None, tol=1e-10, maxit=500, prec=0,
                  scale=1.0, inner_tol=1e-4):
    """Differentiable solve of (A + mu I) x = b with the Nystrom preconditioner P.

    RBF: pass points X and bandwidth sigma (tensor or float); ridge: pass data
    X with kind=1 (A = scale X^T X); dense: pass A.  b, mu and sigma may
    require grad; X may require grad for the ridge form only.
    """
    dev = b.device
    if A is not None:
        data, k = A, OP_DENSE
    elif kind == OP_XTX:
        data, k = X, OP_XTX
    else:
        data, k = X, OP_RBF
        if sigma is None:
            raise ValueError("nystrom_solve: an RBF operator needs sigma")
    mu_t = mu if torch.is_tensor(mu) else torch.tensor(float(mu), dtype=torch.float64, device=dev)
    sig = sigma if sigma is not None else 0.0
    sig_t = sig if torch.is_tensor(sig) else torch.tensor(float(sig), dtype=torch.float64, device=dev)
    return NystromSolve.apply(b, mu_t, sig_t, data, k, P, tol, maxit, prec, scale, inner_tol)


class RbfCross(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, sigma, X, Xv):
        from . import Operator, nys_rbf_cross
        op = Operator.rbf(X.detach(), float(sigma))
        Xv_d = Xv.detach().contiguous()
        v_d = v.detach().reshape(-1).to(torch.float64).contiguous()
        out = nys_rbf_cross(op, Xv_d, v_d)
        ctx.save_for_backward(v_d)
        ctx.op, ctx.Xv = op, Xv_d
        ctx.sigma_shape, ctx.v_shape, ctx.v_dtype = sigma.shape, v.shape, v.dtype
        return out

    @staticmethod
    def backward(ctx, g):
        from . import nys_rbf_cross
        if ctx.needs_input_grad[2] or ctx.needs_input_grad[3]:
            raise NotImplementedError("rbf_cross: gradients with respect to the points are not formed; detach them")
        (v,) = ctx.saved_tensors
        g = g.reshape(-1).to(torch.float64).contiguous()
        gv = (nys_rbf_cross(ctx.op, ctx.Xv, g, transpose=True).reshape(ctx.v_shape).to(ctx.v_dtype)
              if ctx.needs_input_grad[0] else None)
        gsig = None
        if ctx.needs_input_grad[1]:
            _, ds = nys_rbf_cross(ctx.op, ctx.Xv, g, wvec=v)
            gsig = torch.tensor(ds, dtype=torch.float64, device=v.device).reshape(ctx.sigma_shape)
        return gv, gsig, None, None


def rbf_cross(v, sigma, X, Xv):
    """Differentiable u = K(Xv, X; sigma) v (held-out rows of the RBF kernel
    times v); v and sigma may require grad."""
    sig_t = sigma if torch.is_tensor(sigma) else torch.tensor(float(sigma), dtype=torch.float64, device=v.device)
    return RbfCross.apply(v, sig_t, X, Xv)
