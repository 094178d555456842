"""Differentiable receiver misfit: J(c) = 1/2 sum_s ||P u_s - d_s||^2 with A(c) u_s = f_s.

Forward: helm_setup for c, helm_solve for all sources (FGMRES with the recursive sweep),
helm_misfit (J and the adjoint source P^T (P u - d)).  Backward: helm_solve with adjoint = 1
(A^H lam = P^T (P u - d), preconditioned by M^{-H}), then helm_grad_c
(dJ/dc_p = 2 omega^2 / c_p^3 Re sum_s conj(lam_s,p) u_s,p).  Every step runs in libhelm's
kernels; this module only passes tensors.
"""
import torch

from .binding import Helm


class HelmMisfit(torch.autograd.Function):
    """J = HelmMisfit.apply(c, sources, d_obs, plane_k, params) with params a dict holding
    omega, b, C, p, slab_layers, prec, tol, restart, maxit.

    c: float64 CUDA tensor (n, n, n); sources: complex128 (S, n, n, n); d_obs: complex128
    (S, n, n) data on the x3-layer plane_k (1-based).  Returns a float64 scalar tensor.
    params may also hold fronts and fronts_inner (the preconditioner's sweep directions).
    """

    @staticmethod
    def forward(ctx, c, sources, d_obs, plane_k, params):
        H = Helm(c.detach(), params["omega"], params["b"], params["C"], params["p"],
                 params.get("slab_layers", 1), prec=params.get("prec", "c64"),
                 fronts=params.get("fronts", 1), fronts_inner=params.get("fronts_inner", 1))
        tol = params.get("tol", 1e-8)
        restart = params.get("restart", 50)
        maxit = params.get("maxit", 500)
        u, its, rel, rc = H.solve(sources, tol=tol, restart=restart, maxit=maxit)
        J, g = H.misfit(u, d_obs, plane_k)
        ctx.H = H
        ctx.solver = (tol, restart, maxit)
        ctx.forward_iters = its
        ctx.save_for_backward(u, g)
        return torch.tensor(J, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, grad_J):
        u, g = ctx.saved_tensors
        H = ctx.H
        tol, restart, maxit = ctx.solver
        lam, its, rel, rc = H.solve(g, tol=tol, restart=restart, maxit=maxit, adjoint=True)
        grad = H.grad_c(u, lam)
        H.close()
        ctx.H = None
        return grad_J * grad, None, None, None, None


def misfit(c, sources, d_obs, plane_k, **params):
    """Convenience wrapper: HelmMisfit.apply with keyword parameters."""
    return HelmMisfit.apply(c, sources, d_obs, plane_k, params)
