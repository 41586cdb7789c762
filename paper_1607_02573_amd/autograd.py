"""eps -> S as a torch.autograd.Function whose backward is the adjoint solve
(paper Section 5: the gradient needs one more solve with the same operator,
hence the same factors, because A is complex symmetric).

Forward:  A(eps) assembled on the device, subdomains factored, U = A^-1 B
(ports tx), S = conj(P_rx^T U) / nu.
Backward: given dL/dS (PyTorch's convention for a real loss: dL/dRe + i dL/dIm),
one adjoint solve with the factors of the forward pass and a per-tetrahedron
kernel give dL/deps in the same convention.  The adjoint problem must use the
state problem's own operator: if the problem has been updated or refactored
since this forward pass (another forward, a line-search evaluation), its
operator and factors are rebuilt from this pass's eps first.
"""
from __future__ import annotations

import torch


class MaxwellS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, problem, part, n_sub, tx, rx, precision="c128", tol=1e-8, restart=30, maxit=1000):
        e = eps.detach().contiguous()
        problem.update_eps(e)
        problem.factor(part, n_sub, 1, precision)
        Bm = problem.rhs_ports(tx)
        U, _ = problem.solve(Bm, tol=tol, restart=restart, maxit=maxit)
        S = problem.s_matrix(U, rx)
        ctx.problem, ctx.tx, ctx.rx = problem, tx, rx
        ctx.opts = (tol, restart, maxit)
        ctx.setup = (part, n_sub, precision)
        ctx.state = problem.state()
        ctx.save_for_backward(U, e.clone())
        return S

    @staticmethod
    def backward(ctx, gS):
        U, eps = ctx.saved_tensors
        tol, restart, maxit = ctx.opts
        P = ctx.problem
        if P.state() != ctx.state:
            part, n_sub, precision = ctx.setup
            P.update_eps(eps)
            P.factor(part, n_sub, 1, precision)
        g = P.adjoint_gradient(U, gS.contiguous(), ctx.tx, ctx.rx, tol=tol, restart=restart, maxit=maxit)
        return g, None, None, None, None, None, None, None, None, None


def s_of_eps(eps, problem, part, n_sub, tx, rx, **kw):
    return MaxwellS.apply(eps, problem, part, n_sub, tx, rx, kw.get("precision", "c128"), kw.get("tol", 1e-8),
                          kw.get("restart", 30), kw.get("maxit", 1000))
