"""torch.autograd.Function for FWI-style misfits on top of libelh.

Forward model: d_s = P_r u_s with H(lam, mu, rho) u_s = q_s (the mixed
discretization; the solver of Section 5).  P_r samples the wavefield at a
list of receiver storage indices.  The misfit is Phi = 1/2 sum_s |P_r u_s -
d_obs,s|^2.  The backward pass is the adjoint state: with torch's complex
convention dL = Re(g^H dd), the adjoint source is P_r^T g, H^H v_s = P_r^T
g_s, and dL/dm = - Re sum_s v_s^H (dH/dm) u_s, which elh_gradient
evaluates.  Solves, receiver sampling, misfit and injection all run in the
HIP library.
"""
import torch

from .api import Problem


def _indices(problem, receivers):
    """receiver storage indices from an int64 index vector or a bool mask"""
    if receivers.dtype == torch.bool:
        return problem.receiver_indices(receivers)
    return problem._idx(receivers)


def _forward(problem, lam, mu, rho, q, rtol, maxit):
    problem.set_media(lam.detach(), mu.detach(), rho.detach())
    u, info, code = problem.solve(q.contiguous(), rtol=rtol, maxit=maxit)
    if code != 0:
        raise RuntimeError("forward solve did not converge: %s" % info)
    return u


def _adjoint(problem, u, grad_src, rtol, maxit):
    v, info, code = problem.solve_adjoint(grad_src, rtol=rtol, maxit=maxit)
    if code != 0:
        raise RuntimeError("adjoint solve did not converge: %s" % info)
    return problem.gradient(u, v)


class ElasticFWI(torch.autograd.Function):
    """d = ElasticFWI.apply(lam, mu, rho, problem, q, idx, rtol, maxit)

    lam, mu, rho: float64 CUDA tensors (numpy grid shape); problem: a
    Problem whose media are replaced by (lam, mu, rho); q: complex128
    sources (nrhs, d+1, ...); idx: int64 receiver storage indices (see
    Problem.receiver_indices).  Returns the receiver data (nrhs, nrec).
    The problem's media stay at (lam, mu, rho) until the next forward call,
    so call backward before re-using the problem.
    """

    @staticmethod
    def forward(ctx, lam, mu, rho, problem, q, idx, rtol=1e-10, maxit=1000):
        u = _forward(problem, lam, mu, rho, q, rtol, maxit)
        ctx.problem, ctx.rtol, ctx.maxit = problem, rtol, maxit
        ctx.save_for_backward(u, idx)
        return problem.receivers(u, idx)

    @staticmethod
    def backward(ctx, grad_d):
        u, idx = ctx.saved_tensors
        problem = ctx.problem
        src = problem.inject(grad_d.to(torch.complex128).contiguous(), idx)
        g_lam, g_mu, g_rho = _adjoint(problem, u, src, ctx.rtol, ctx.maxit)
        return g_lam, g_mu, g_rho, None, None, None, None, None


class ElasticMisfit(torch.autograd.Function):
    """phi = ElasticMisfit.apply(lam, mu, rho, problem, q, idx, d_obs, rtol,
    maxit): the total misfit 1/2 sum_s |P_r u_s - d_obs,s|^2 (a 0-d float64
    tensor); d_obs: (nrhs, nrec) complex128 receiver data."""

    @staticmethod
    def forward(ctx, lam, mu, rho, problem, q, idx, d_obs, rtol=1e-10, maxit=1000):
        u = _forward(problem, lam, mu, rho, q, rtol, maxit)
        r, phi = problem.receivers(u, idx, d_obs.contiguous(), misfit=True)
        ctx.problem, ctx.rtol, ctx.maxit = problem, rtol, maxit
        ctx.save_for_backward(u, idx, r)
        return phi[-1]

    @staticmethod
    def backward(ctx, grad_phi):
        u, idx, r = ctx.saved_tensors
        problem = ctx.problem
        # dPhi/dd = r (torch's convention); the chain rule scales it by grad_phi
        src = problem.inject(r, idx, scale=float(grad_phi))
        g_lam, g_mu, g_rho = _adjoint(problem, u, src, ctx.rtol, ctx.maxit)
        return g_lam, g_mu, g_rho, None, None, None, None, None, None


def misfit(problem, lam, mu, rho, q, receivers, d_obs, rtol=1e-10, maxit=1000):
    """Phi = 1/2 sum |P_r u - d_obs|^2 (differentiable in lam, mu, rho).

    receivers: int64 storage indices or a bool mask of the vector's shape;
    d_obs: receiver data (nrhs, nrec), or full wavefields (nrhs, d+1, ...)
    that are sampled at the receivers first."""
    idx = _indices(problem, receivers)
    q = q.contiguous()
    if d_obs.dim() == q.dim():
        d_obs = problem.receivers(d_obs.contiguous(), idx)
    return ElasticMisfit.apply(lam, mu, rho, problem, q, idx, d_obs, rtol, maxit)
