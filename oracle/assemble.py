"""Element matrices, sparse assembly and boundary conditions (oracle; test
infrastructure only).

Section 2, the mixed variational problem and its Taylor-Hood discretisation:
  a(u,v) = int mu grad u : grad v + gamma rho u.v        (bilinear form a)
  b(v,q) = - int q div v                                  (bilinear form b)
  <F,v>  = int f.v                                        (load functional)
giving K = [A B^T; B -C] of the saddle-point system in Section 1, here with the
optional stabilisation C = c_p M_p (Section 1 allows C >= 0; every workload in
use has c_p = 0).

Reading of the sign of b: the paper prints b(u,q) = +int q div u in Section 2
but b_tau(v,q) = -int q div v in Appendix A and in the smoothing analysis of
Section 3.3.2 (integration by parts step).  With the minus sign the first
equation of the mixed problem is -mu Laplace u + grad p = f, i.e. the strong
form (1)-(2) with the physical pressure, so B = -div is used.  The velocity
solution does not depend on this choice.

Deformation-rate form (Sec. 2, used in some applications in place of a):
  a_eps(u,v) = int mu eps(u) : eps(v) + gamma rho u.v,  eps(u) = (grad u + grad u^T) / 2,
as printed (no factor 2 in front of mu).  For the test function phi_i e_d and
the trial function phi_j e_c, eps(u):eps(v) = (delta_cd grad phi_i . grad phi_j
+ d_c phi_i d_d phi_j) / 2, so the velocity block couples the components.

Dirichlet reading: every velocity node on the box boundary is constrained;
the constrained matrix has those rows and columns zeroed and a unit diagonal,
so K acts as the identity on constrained entries.

Everything is plain: per-cell quadrature with explicit Lagrange bases and the
multilinear geometry map (Jacobian J, det J, J^{-1}), COO triplets summed into
CSR by scipy.
"""
import numpy as np
import scipy.sparse as sp

from .fe import gauss_rule, gll_points, reference_basis, quadrature_weights, tensor_multi_indices
from .mesh import multilinear_shape_grad


class CellData:
    """Quadrature-point geometry and basis data for a list of cells."""

    def __init__(self, mesh, cells, nq_1d=None):
        d, k = mesh.dim, mesh.k
        nq_1d = k + 1 if nq_1d is None else nq_1d
        xq, wq = gauss_rule(nq_1d)
        qid = tensor_multi_indices(nq_1d, d)
        xi = xq[qid]                                               # (nq, d)
        self.w = quadrature_weights(wq, d)
        self.phi, dphi_ref = reference_basis(gll_points(k + 1), d, xq)   # (nv, nq), (nv, nq, d)
        self.psi, _ = reference_basis(gll_points(k), d, xq)              # (np, nq)
        X = mesh.vertices[mesh.cell_vertex_ids(cells)]            # (nc, 2^d, d)
        dN = multilinear_shape_grad(xi, d)                        # (nq, 2^d, d)
        J = np.einsum("cva,qvb->cqab", X, dN)                     # dx_a / dxi_b
        self.detJ = np.linalg.det(J)
        if np.any(self.detJ <= 0):
            raise ValueError("degenerate or inverted cell")
        Jinv = np.linalg.inv(J)                                   # dxi_b / dx_a
        # physical gradients: grad_x phi_a = sum_b dphi/dxi_b * dxi_b/dx_a
        self.grad = np.einsum("iqb,cqba->ciqa", dphi_ref, Jinv)   # (nc, nv, nq, d)
        self.JxW = self.detJ * self.w[None, :]
        self.xq = np.einsum("qv,cva->cqa", _mlin(xi, d), X)       # physical quadrature points


def _mlin(xi, d):
    from .mesh import multilinear_shape
    return multilinear_shape(xi, d)


def element_matrices(mesh, cells, mu, gamma, rho):
    """Per-cell matrices for the cells `cells`:
      A_tau[c, i, j]       = int mu grad phi_i . grad phi_j + gamma rho phi_i phi_j
      B_tau[c, i, comp, j] = - int psi_i d(phi_j)/dx_comp
      Mp_tau[c, i, j]      = int psi_i psi_j
      Mv_tau[c, i, j]      = int phi_i phi_j
    with mu an array over the cells."""
    cd = CellData(mesh, cells)
    mu = np.asarray(mu, dtype=np.float64)
    stiff = np.einsum("ciqa,cjqa,cq->cij", cd.grad, cd.grad, cd.JxW)
    mass_v = np.einsum("iq,jq,cq->cij", cd.phi, cd.phi, cd.JxW)
    A = mu[:, None, None] * stiff + (gamma * rho) * mass_v
    B = -np.einsum("iq,cjqa,cq->ciaj", cd.psi, cd.grad, cd.JxW)
    Mp = np.einsum("iq,jq,cq->cij", cd.psi, cd.psi, cd.JxW)
    return A, B, Mp, mass_v


def symmetric_gradient_blocks(mesh, cells, mu, gamma, rho):
    """Per-cell velocity blocks of a_eps: out[c, d, i, e, j] = a_eps(phi_j e_e, phi_i e_d)
      = mu/2 (delta_de int grad phi_i . grad phi_j + int d_e phi_i d_d phi_j)
        + gamma rho delta_de int phi_i phi_j."""
    cd = CellData(mesh, cells)
    d = mesh.dim
    mu = np.asarray(mu, dtype=np.float64)
    G = np.einsum("ciqa,cjqb,cq->ciajb", cd.grad, cd.grad, cd.JxW)       # int d_a phi_i d_b phi_j
    stiff = np.einsum("ciaja->cij", G)
    mass_v = np.einsum("iq,jq,cq->cij", cd.phi, cd.phi, cd.JxW)
    nc, nv = stiff.shape[0], stiff.shape[1]
    out = np.zeros((nc, d, nv, d, nv))
    for dt in range(d):
        for ct in range(d):
            blk = 0.5 * G[:, :, ct, :, dt]
            if dt == ct:
                blk = blk + 0.5 * stiff
            out[:, dt, :, ct, :] = mu[:, None, None] * blk + (gamma * rho * mass_v if dt == ct else 0.0)
    return out


class Assembled:
    """The constrained sparse system of one level.

    Attributes: A (d Nv square, block diagonal over components), B (Np x d Nv),
    Mp, Mv (unconstrained velocity mass, one component), K (full saddle-point
    matrix), constrained (global indices), plus the per-cell matrices needed by
    the local Schur diagonal."""

    def __init__(self, mesh, mu=1.0, gamma=0.0, rho=1.0, c_p=0.0, chunk=4096, keep_local=True, form="grad"):
        if form not in ("grad", "sym"):
            raise ValueError(form)
        self.form = form
        d = mesh.dim
        Nv, Np = mesh.n_vnode, mesh.n_pnode
        self.mesh = mesh
        self.gamma, self.rho, self.c_p = gamma, rho, c_p
        mu_cell = mesh.mu(mu)
        rA, cA, vA = [], [], []
        rB, cB, vB = [], [], []
        rM, cM, vM = [], [], []
        rV, cV, vV = [], [], []
        local_Adiag, local_B = [], []
        for s in range(0, mesh.ncell, chunk):
            cells = np.arange(s, min(s + chunk, mesh.ncell))
            A_t, B_t, Mp_t, Mv_t = element_matrices(mesh, cells, mu_cell[cells], gamma, rho)
            vn = mesh.cell_velocity_nodes(cells)                  # (nc, nv)
            pn = mesh.cell_pressure_nodes(cells)                  # (nc, np)
            nv, npl = vn.shape[1], pn.shape[1]
            if form == "sym":
                Ablk = symmetric_gradient_blocks(mesh, cells, mu_cell[cells], gamma, rho)   # (nc, d, nv, d, nv)
                for dt in range(d):          # test component
                    for ct in range(d):      # trial component
                        rA.append(np.repeat(vn + dt * Nv, nv, axis=1).ravel())
                        cA.append(np.tile(vn + ct * Nv, (1, nv)).ravel())
                        vA.append(Ablk[:, dt, :, ct, :].ravel())
            for comp in range(d):
                g = vn + comp * Nv
                if form == "grad":
                    rA.append(np.repeat(g, nv, axis=1).ravel())
                    cA.append(np.tile(g, (1, nv)).ravel())
                    vA.append(A_t.ravel())
                rB.append(np.repeat(pn, nv, axis=1).ravel())
                cB.append(np.tile(g, (1, npl)).ravel())
                vB.append(B_t[:, :, comp, :].ravel())
            rM.append(np.repeat(pn, npl, axis=1).ravel())
            cM.append(np.tile(pn, (1, npl)).ravel())
            vM.append(Mp_t.ravel())
            rV.append(np.repeat(vn, nv, axis=1).ravel())
            cV.append(np.tile(vn, (1, nv)).ravel())
            vV.append(Mv_t.ravel())
            if keep_local and form == "grad":
                local_Adiag.append(np.einsum("cii->ci", A_t))
                local_B.append(B_t)
        cat = np.concatenate
        A = sp.coo_matrix((cat(vA), (cat(rA), cat(cA))), shape=(d * Nv, d * Nv)).tocsr()
        B = sp.coo_matrix((cat(vB), (cat(rB), cat(cB))), shape=(Np, d * Nv)).tocsr()
        self.Mp = sp.coo_matrix((cat(vM), (cat(rM), cat(cM))), shape=(Np, Np)).tocsr()
        self.Mv = sp.coo_matrix((cat(vV), (cat(rV), cat(cV))), shape=(Nv, Nv)).tocsr()
        self.A_unconstrained = A
        self.B_unconstrained = B
        # Dirichlet: zero rows and columns, unit diagonal on constrained DoFs
        self.constrained = mesh.constrained_dofs()
        free = np.ones(d * Nv)
        free[self.constrained] = 0.0
        Dfree = sp.diags(free)
        Dcon = sp.diags(1.0 - free)
        self.A = (Dfree @ A @ Dfree + Dcon).tocsr()
        self.B = (B @ Dfree).tocsr()
        self.free_u = free
        self.C = (c_p * self.Mp).tocsr()
        self.K = sp.bmat([[self.A, self.B.T], [self.B, -self.C]]).tocsr()
        if keep_local and form == "grad":
            self.local_Adiag = cat(local_Adiag)                   # (ncell, nv)
            self.local_B = cat(local_B, axis=0)                   # (ncell, np, d, nv)

    # --- vector helpers --------------------------------------------------
    def split(self, x):
        nu = self.A.shape[0]
        return x[:nu], x[nu:]

    def rhs_from_nodal_f(self, f_nodal):
        """b = [M_v f_1, ..., M_v f_d, 0] with the constrained entries set to 0
        (load functional <F, v> of Section 2 for a nodal FE field f)."""
        d = self.mesh.dim
        Nv = self.mesh.n_vnode
        f = np.asarray(f_nodal, dtype=np.float64).reshape(d, Nv)
        bu = np.concatenate([self.Mv @ f[c] for c in range(d)])
        bu *= self.free_u
        return np.concatenate([bu, np.zeros(self.mesh.n_pnode)])


def rhs_closed_form(mesh, f, extra_q=2):
    """b_u,i = sum_tau sum_q f(x_q) . phi_i(x_q) JxW_q with k+1+extra_q Gauss
    points per direction; b_p = 0; constrained entries 0."""
    d = mesh.dim
    Nv = mesh.n_vnode
    cells = np.arange(mesh.ncell)
    cd = CellData(mesh, cells, nq_1d=mesh.k + 1 + extra_q)
    fq = f(cd.xq.reshape(-1, d)).reshape(len(cells), -1, d)   # (nc, nq, d)
    loc = np.einsum("iq,cqa,cq->cai", cd.phi, fq, cd.JxW)
    vn = mesh.cell_velocity_nodes(cells)
    bu = np.zeros((d, Nv))
    for comp in range(d):
        np.add.at(bu[comp], vn.ravel(), loc[:, comp, :].ravel())
    bu = bu.ravel()
    bu[mesh.constrained_dofs()] = 0.0
    return np.concatenate([bu, np.zeros(mesh.n_pnode)])
