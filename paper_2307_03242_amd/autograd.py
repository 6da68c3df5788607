"""torch.autograd.Function for FWI-style misfits on top of libelh.

Forward model: d_s = P_r u_s with H(lam, mu, rho) u_s = q_s (eq.
mixed-discretized; the solver of Section 5).  P_r samples the vector at a
boolean receiver mask (storage layout).  The backward pass is the adjoint
state: with torch's complex convention dL = Re(g^H dd), the adjoint source
is P_r^T g, H^H v_s = P_r^T g_s, and dL/dm = - Re sum_s v_s^H (dH/dm) u_s,
which elh_gradient evaluates.  All numerical work runs in the HIP library.
"""
import torch

from .api import Problem


class ElasticFWI(torch.autograd.Function):
    """d = ElasticFWI.apply(lam, mu, rho, problem, q, mask, rtol, maxit)

    lam, mu, rho: float64 CUDA tensors (numpy grid shape); problem: a
    Problem whose media are replaced by (lam, mu, rho); q: complex128
    sources (nrhs, d+1, ...); mask: bool tensor (d+1, ...) of receivers.
    Returns the masked wavefields (nrhs, d+1, ...), zero off the receivers.
    The problem's media stay at (lam, mu, rho) until the next forward call,
    so call backward before re-using the problem.
    """

    @staticmethod
    def forward(ctx, lam, mu, rho, problem, q, mask, rtol=1e-10, maxit=1000):
        problem.set_media(lam.detach(), mu.detach(), rho.detach())
        u, info, code = problem.solve(q.contiguous(), rtol=rtol, maxit=maxit)
        if code != 0:
            raise RuntimeError("forward solve did not converge: %s" % info)
        ctx.problem, ctx.rtol, ctx.maxit = problem, rtol, maxit
        ctx.save_for_backward(u, mask)
        return u * mask

    @staticmethod
    def backward(ctx, grad_d):
        u, mask = ctx.saved_tensors
        problem = ctx.problem
        r = (grad_d * mask).to(torch.complex128).contiguous()
        v, info, code = problem.solve_adjoint(r, rtol=ctx.rtol, maxit=ctx.maxit)
        if code != 0:
            raise RuntimeError("adjoint solve did not converge: %s" % info)
        g_lam, g_mu, g_rho = problem.gradient(u, v)
        return g_lam, g_mu, g_rho, None, None, None, None, None


def misfit(problem, lam, mu, rho, q, mask, d_obs, rtol=1e-10, maxit=1000):
    """Phi = 1/2 sum |P_r u - d_obs|^2 (differentiable in lam, mu, rho)."""
    d = ElasticFWI.apply(lam, mu, rho, problem, q, mask, rtol, maxit)
    r = d - d_obs * mask
    return 0.5 * (r.abs() ** 2).sum()
