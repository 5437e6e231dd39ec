"""Differentiable Stokes solve.

`solve(f, log_mu, **problem)` returns the finest-level solution x = [u | p]
of K(mu) x = [Z M_v f; 0] (mu = exp(log_mu) per finest cell, f a nodal
velocity field) as a torch tensor that autograd can differentiate with
respect to f and log_mu.  The backward pass is the adjoint solve K lam = dJ/dx
with the same symmetric operator and multigrid preconditioner (smg_solve;
K = K^T), followed by the adjoint-state gradients of smg_gradient:
  dJ/d log mu_tau = -mu_tau int_tau grad lam_u : grad u,   dJ/df = M_v Z lam_u.
All arithmetic runs in the library's kernels; this module only orders the
calls (a fresh hierarchy is set up for each viscosity field, since the
diagonals, eigenvalue bounds and the coarse inverse depend on mu).
"""
import torch

from . import StokesMG, SMG_BLOCK_MASS


class StokesSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, log_mu, problem, rtol, maxit):
        mu = torch.exp(log_mu.detach()).cpu().numpy()
        mg = StokesMG(mu_cell=mu, **problem)
        L = mg.n_levels - 1
        nu, np_ = mg.sizes(L)
        b = torch.zeros(nu + np_, dtype=torch.float64, device=f.device)
        mg.apply_block(L, SMG_BLOCK_MASS, f.detach().to(torch.float64).contiguous(), b[:nu])
        x = torch.zeros_like(b)
        mg.solve(x, b, rtol=rtol, maxit=maxit)
        ctx.mg, ctx.rtol, ctx.maxit = mg, rtol, maxit
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        mg = ctx.mg
        g = gx.detach().to(torch.float64).contiguous().clone()
        # for C = 0 the returned pressure is normalised to M_p-weighted mean
        # zero; the transpose of that map (a library call, which leaves g as
        # it is for C != 0, where nothing is normalised) makes the adjoint
        # right-hand side orthogonal to the constant pressure
        mg.pressure_mean_adjoint(g)
        lam = torch.zeros_like(g)
        if torch.count_nonzero(g) > 0:
            mg.solve(lam, g, rtol=ctx.rtol, maxit=ctx.maxit)
        g_logmu, g_f = mg.gradient(x, lam, want_logmu=ctx.needs_input_grad[1], want_f=ctx.needs_input_grad[0])
        mg.close()
        ctx.mg = None
        return g_f, g_logmu, None, None, None


def solve(f, log_mu, rtol=1e-10, maxit=300, **problem):
    """Differentiable solve; `problem` holds the StokesMG arguments other than
    mu_cell (dim, fe_degree, n_coarse, n_levels, fine_vertices, gamma, ...)."""
    return StokesSolve.apply(f, log_mu, problem, rtol, maxit)
