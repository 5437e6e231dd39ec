"""Grid transfer (oracle; test infrastructure only).

Section 3.2: the prolongation I_{l-1}^l is the matrix of the canonical
injection V_{l-1} x Q_{l-1} -> V_l x Q_l, and the restriction is its
transpose.  Written out: P[i, j] = phi_j^{(l-1)}(x_i^{(l)}), each coarse basis
function evaluated at each fine node, field by field (velocity components
and pressure separately).  The evaluation uses reference-lattice coordinates,
which is the injection itself on nested (e.g. Cartesian) meshes and the
reading used on perturbed hierarchies.  Constrained (Dirichlet) fine rows and
coarse columns are zero.
"""
import numpy as np
import scipy.sparse as sp

from .fe import gll_points, lagrange_values


def _field_prolongation(n_coarse, deg, dim):
    """P for one scalar Q_deg field on the box lattice, fine = 2 * coarse."""
    z = gll_points(deg + 1)
    n_f = [2 * v for v in n_coarse]
    dims_f = [deg * v + 1 for v in n_f]
    dims_c = [deg * v + 1 for v in n_coarse]
    nfine = int(np.prod(dims_f))
    fine = np.arange(nfine, dtype=np.int64)
    # per-direction: coarse cell of each fine node and the position in it
    lat = []
    rem = fine.copy()
    for a in range(dim):
        lat.append(rem % dims_f[a])
        rem //= dims_f[a]
    rows, cols, vals = [], [], []
    per_dir = []
    for a in range(dim):
        I = lat[a]
        cf = np.minimum(I // deg, n_f[a] - 1)
        xi_f = z[I - cf * deg]
        cc = cf // 2
        xi_c = (cf - 2 * cc + xi_f) / 2.0
        Vals = lagrange_values(z, xi_c).T                     # (nfine, deg+1)
        per_dir.append((cc, Vals))
    loc = np.indices((deg + 1,) * dim).reshape(dim, -1)[::-1].T
    for off in loc:
        w = np.ones(nfine)
        col = np.zeros(nfine, dtype=np.int64)
        stride = 1
        for a in range(dim):
            cc, Vals = per_dir[a]
            w *= Vals[:, off[a]]
            col += (deg * cc + off[a]) * stride
            stride *= dims_c[a]
        rows.append(fine)
        cols.append(col)
        vals.append(w)
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nfine, int(np.prod(dims_c)))).tocsr()
    P.eliminate_zeros()
    return P


def prolongation(mesh_coarse, mesh_fine):
    """Block-diagonal P over [u_1 | ... | u_d | p] with Dirichlet rows/columns zero."""
    d, k = mesh_fine.dim, mesh_fine.k
    assert all(2 * a == b for a, b in zip(mesh_coarse.n, mesh_fine.n))
    Pv = _field_prolongation(mesh_coarse.n, k, d)
    Pp = _field_prolongation(mesh_coarse.n, k - 1, d)
    fr = (~mesh_fine.velocity_boundary_nodes()).astype(np.float64)
    cc = (~mesh_coarse.velocity_boundary_nodes()).astype(np.float64)
    Pv = (sp.diags(fr) @ Pv @ sp.diags(cc)).tocsr()
    Pv.eliminate_zeros()
    return sp.block_diag([Pv] * d + [Pp], format="csr")


def restriction(mesh_coarse, mesh_fine):
    return prolongation(mesh_coarse, mesh_fine).T.tocsr()
