"""Adjoint-state gradients of a solve (oracle; test infrastructure only).

The discrete saddle-point system of Section 1, K(mu) x = b(f), with
b = [Z M_v f; 0] (nodal force field f, Z zeroing the constrained velocity
rows), is symmetric (K = K^T; the Dirichlet rows and columns are the
identity).  For an objective J(x) the adjoint state lam solves K lam = dJ/dx
and, since K depends on the per-cell viscosity only through the first term of
the form a of Section 2 (mu_tau int_tau grad u : grad v, or mu_tau int_tau
eps(u) : eps(v) for the deformation-rate form, where A_tau^grad below is that
form's cell matrix at unit viscosity),

  dJ/d log mu_tau = - mu_tau  lam_u^T A_tau^grad u     (constrained entries zeroed),
  dJ/df           = M_v^T Z lam_u = M_v (Z lam_u)      (per component, every node),

with A_tau^grad the cell stiffness matrix int_tau grad phi_i . grad phi_j.
Everything here is assembled from the same per-cell quadrature as
`assemble.element_matrices`, and the solves are direct (sparse LU of the
bordered system that fixes the pressure mean).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import element_matrices, symmetric_gradient_blocks


def bordered_solve(asm, rhs):
    """x with K x = rhs and M_p-weighted pressure mean zero (the bordered
    system [K m; m^T 0] of the coarse solve, here on any level)."""
    nu = asm.A.shape[0]
    n = asm.K.shape[0]
    m = np.zeros(n)
    m[nu:] = asm.Mp @ np.ones(n - nu)
    Kb = sp.bmat([[asm.K, sp.csr_matrix(m[:, None])], [sp.csr_matrix(m[None, :]), None]]).tocsc()
    return spla.spsolve(Kb, np.concatenate([rhs, [0.0]]))[:-1]


def state_solve(asm, rhs):
    """The solution map of Section 2's discrete problem: for C = 0 the
    pressure is fixed up to a constant and the bordered solve above returns
    the one with M_p-weighted mean zero; for C = c_p M_p, c_p > 0, K is
    regular and solved as it is."""
    if asm.c_p == 0.0:
        return bordered_solve(asm, rhs)
    return spla.spsolve(asm.K.tocsc(), rhs)


def normalisation_adjoint(asm, g):
    """Transpose of the pressure normalisation p <- p - 1 (m.p)/(m.1), m =
    M_p 1, applied to an adjoint right-hand side g (velocity block
    unchanged): g_p <- g_p - m (1.g_p)/(m.1).  Identity for C != 0, where the
    solution is not normalised."""
    if asm.c_p != 0.0:
        return g.copy()
    nu = asm.A.shape[0]
    m = asm.Mp @ np.ones(asm.Mp.shape[0])
    out = g.copy()
    out[nu:] = g[nu:] - m * (g[nu:].sum() / m.sum())
    return out


def rhs_from_force(asm, f_nodal):
    """b = [Z M_v f; 0] for a nodal velocity field f of shape (d, Nv)."""
    return asm.rhs_from_nodal_f(np.asarray(f_nodal).reshape(asm.mesh.dim, -1))


def velocity_objective(asm, x, u_target):
    """J = sum over velocity DoFs of (u - u_target)^2, and dJ/dx."""
    nu = asm.A.shape[0]
    du = x[:nu] - u_target
    g = np.zeros_like(x)
    g[:nu] = 2.0 * du
    return float(du @ du), g


def gradients(asm, x, lam):
    """(dJ/d log mu per cell, dJ/df per velocity DoF) from the state x and the
    adjoint state lam of the constrained system."""
    mesh = asm.mesh
    d = mesh.dim
    Nv = mesh.n_vnode
    free = asm.free_u
    u = x[:d * Nv] * free
    lu = lam[:d * Nv] * free
    mu = mesh.mu(1.0)
    cells = np.arange(mesh.ncell)
    vn = mesh.cell_velocity_nodes(cells)
    g_mu = np.zeros(mesh.ncell)
    if asm.form == "sym":
        # the viscous part of the deformation-rate form at unit viscosity
        blk = symmetric_gradient_blocks(mesh, cells, np.ones(mesh.ncell), 0.0, 1.0)   # (nc, d, nv, d, nv)
        U = np.stack([u[c * Nv:(c + 1) * Nv][vn] for c in range(d)], axis=1)        # (nc, d, nv)
        Lm = np.stack([lu[c * Nv:(c + 1) * Nv][vn] for c in range(d)], axis=1)
        g_mu -= np.einsum("cdi,cdiej,cej->c", Lm, blk, U)
    else:
        stiff, _, _, _ = element_matrices(mesh, cells, np.ones(mesh.ncell), 0.0, 1.0)
        for c in range(d):
            uc = u[c * Nv:(c + 1) * Nv][vn]           # (nc, nv)
            lc = lu[c * Nv:(c + 1) * Nv][vn]
            g_mu -= np.einsum("ci,cij,cj->c", lc, stiff, uc)
    g_mu *= mu
    g_f = np.concatenate([asm.Mv @ lu[c * Nv:(c + 1) * Nv] for c in range(d)])
    return g_mu, g_f
