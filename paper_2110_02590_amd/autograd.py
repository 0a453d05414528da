"""The reduced AL objective as a torch.autograd.Function.

phi(u) = sigma_f f(x(u), u) + y^T D_c (c(x(u), u) - s) + rho/2 ||D_c (c - s)||^2
with x(u) the power-flow solution (Section III-A).  forward solves the
power flow and evaluates phi; backward multiplies the reduced gradient
(Proposition 1, the library's adjoint kernels) by grad_output.  The gradient
is itself a Function whose backward is the reduced Hessian-vector product
(Proposition 2): differentiating the gradient again (forward-over-reverse)
runs the adjoint-adjoint kernels.  H is symmetric, so vjp = jvp = H v.
All arithmetic runs in the HIP library; this module only routes tensors.
"""
from __future__ import annotations

import torch


class _Ctx:
    """Problem data shared by the two Functions (not differentiated)."""

    def __init__(self, problem, s, y, rho, sigma, pd=None, qd=None, tol=1e-10, max_iter=20):
        self.pr = problem
        self.s, self.y, self.rho, self.sigma = s, y, float(rho), sigma
        self.pd = problem.pd if pd is None else pd
        self.qd = problem.qd if qd is None else qd
        self.tol, self.max_iter = tol, max_iter
        self.x = problem.flat_x()

    def solve(self, u):
        g = self.pr.grid
        st, res = g.pf_solve(u, self.pd, self.qd, self.x, tol=self.tol, max_iter=self.max_iter)
        if int(st[1]) != 1:
            raise RuntimeError(f"power flow did not converge (residual {float(res):.3e})")
        return self.x.clone()


class ReducedALGrad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, x, C):
        grad, _ = C.pr.grid.reduced_gradient(x, u.contiguous(), C.pd, C.qd, C.s, C.y, C.rho, C.sigma)
        ctx.C = C
        ctx.save_for_backward(u, x)
        return grad

    @staticmethod
    def backward(ctx, v):
        u, x = ctx.saved_tensors
        C = ctx.C
        g = C.pr.grid
        # the handle caches one point: refresh it for (x, u)
        g.reduced_gradient(x, u.contiguous(), C.pd, C.qd, C.s, C.y, C.rho, C.sigma)
        hv = g.hessian_batch(v.detach().reshape(-1, 1).contiguous().to(torch.float64)).reshape(-1)
        return hv, None, None


class ReducedAL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, C):
        x = C.solve(u.detach().contiguous())
        phi, _ = C.pr.grid.al_objective(x, u.contiguous(), C.pd, C.qd, C.s, C.y, C.rho, C.sigma)
        ctx.C = C
        ctx.save_for_backward(u, x)
        return phi.reshape(())

    @staticmethod
    def backward(ctx, gout):
        u, x = ctx.saved_tensors
        grad = ReducedALGrad.apply(u, x, ctx.C)
        return gout * grad, None


def reduced_al(u, problem, s, y, rho, sigma, **kw):
    """phi(u) with autograd support; see the module docstring."""
    return ReducedAL.apply(u, _Ctx(problem, s, y, rho, sigma, **kw))
