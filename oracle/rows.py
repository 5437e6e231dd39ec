"""Single rows of K x at any mesh size (oracle; test infrastructure only).

(K x)_i of the constrained saddle-point matrix of Section 2, computed from the
definition K x = sum_tau P_tau K_tau P_tau^T x (Section 3.1) restricted to
the cells that contain DoF i: the element matrices of those cells come from
the same quadrature as the assembled oracle.  Used where the full matrix is
too large to assemble (sampled checks at full workload size).
"""
import numpy as np

from .assemble import element_matrices


def _cells_touching(mesh, lat, deg):
    """Cells (flat ids) containing the lattice node `lat` of a Q_deg field."""
    d = mesh.dim
    options = []
    for a in range(d):
        i = int(lat[a])
        c = i // deg
        cand = []
        if i % deg == 0:
            if c - 1 >= 0:
                cand.append(c - 1)
            if c <= mesh.n[a] - 1:
                cand.append(c)
        else:
            cand.append(c)
        options.append(cand)
    cells = []
    for ia in options[0]:
        for ib in options[1]:
            if d == 2:
                cells.append(ia + mesh.n[0] * ib)
            else:
                for ic in options[2]:
                    cells.append(ia + mesh.n[0] * (ib + mesh.n[1] * ic))
    return cells


def sample_Kx(mesh, x, dofs, mu=1.0, gamma=0.0, rho=1.0, c_p=0.0):
    d, k = mesh.dim, mesh.k
    Nv, Np = mesh.n_vnode, mesh.n_pnode
    x = np.asarray(x, dtype=np.float64)
    u = x[:d * Nv].reshape(d, Nv)
    p = x[d * Nv:]
    bnd = mesh.velocity_boundary_nodes()
    mu_cell = mesh.mu(mu)
    uf = u * (~bnd)[None, :]
    out = np.zeros(len(dofs))
    for n_i, g in enumerate(dofs):
        g = int(g)
        if g < d * Nv:
            comp, node = divmod(g, Nv)
            if bnd[node]:
                out[n_i] = x[g]
                continue
            lat = mesh._unflat(np.array([node]), mesh.vel_dims)[0]
            cells = np.array(_cells_touching(mesh, lat, k))
            A_t, B_t, Mp_t, _ = element_matrices(mesh, cells, mu_cell[cells], gamma, rho)
            vn = mesh.cell_velocity_nodes(cells)
            pn = mesh.cell_pressure_nodes(cells)
            s = 0.0
            for c in range(len(cells)):
                li = int(np.nonzero(vn[c] == node)[0][0])
                s += A_t[c, li, :] @ uf[comp, vn[c]]
                s += B_t[c, :, comp, li] @ p[pn[c]]
            out[n_i] = s
        else:
            node = g - d * Nv
            lat = mesh._unflat(np.array([node]), mesh.p_dims)[0]
            cells = np.array(_cells_touching(mesh, lat, k - 1))
            A_t, B_t, Mp_t, _ = element_matrices(mesh, cells, mu_cell[cells], gamma, rho)
            vn = mesh.cell_velocity_nodes(cells)
            pn = mesh.cell_pressure_nodes(cells)
            s = 0.0
            for c in range(len(cells)):
                li = int(np.nonzero(pn[c] == node)[0][0])
                for comp in range(d):
                    s += B_t[c, li, comp, :] @ uf[comp, vn[c]]
                s -= c_p * (Mp_t[c, li, :] @ p[pn[c]])
            out[n_i] = s
    return out


def sample_abs_Kx(mesh, x, dofs, mu=1.0, gamma=0.0, rho=1.0, c_p=0.0):
    """(|K| |x|)_i at the DoFs `dofs`: the entries K_ij of each sampled row
    are summed over the cells around DoF i (per global column j), then
    sum_j |K_ij| |x_j|.  The scale of the componentwise error measure
    |y - K x|_i / (|K| |x|)_i of a computed y."""
    d, k = mesh.dim, mesh.k
    Nv = mesh.n_vnode
    x = np.asarray(x, dtype=np.float64)
    bnd = mesh.velocity_boundary_nodes()
    mu_cell = mesh.mu(mu)
    out = np.zeros(len(dofs))
    for n_i, g in enumerate(dofs):
        g = int(g)
        row = {}
        if g < d * Nv:
            comp, node = divmod(g, Nv)
            if bnd[node]:
                out[n_i] = abs(x[g])
                continue
            lat = mesh._unflat(np.array([node]), mesh.vel_dims)[0]
            cells = np.array(_cells_touching(mesh, lat, k))
            A_t, B_t, _, _ = element_matrices(mesh, cells, mu_cell[cells], gamma, rho)
            vn = mesh.cell_velocity_nodes(cells)
            pn = mesh.cell_pressure_nodes(cells)
            for c in range(len(cells)):
                li = int(np.nonzero(vn[c] == node)[0][0])
                for j, col in enumerate(vn[c]):
                    if not bnd[col]:
                        key = comp * Nv + int(col)
                        row[key] = row.get(key, 0.0) + A_t[c, li, j]
                for j, col in enumerate(pn[c]):
                    key = d * Nv + int(col)
                    row[key] = row.get(key, 0.0) + B_t[c, j, comp, li]
        else:
            node = g - d * Nv
            lat = mesh._unflat(np.array([node]), mesh.p_dims)[0]
            cells = np.array(_cells_touching(mesh, lat, k - 1))
            A_t, B_t, Mp_t, _ = element_matrices(mesh, cells, mu_cell[cells], gamma, rho)
            vn = mesh.cell_velocity_nodes(cells)
            pn = mesh.cell_pressure_nodes(cells)
            for c in range(len(cells)):
                li = int(np.nonzero(pn[c] == node)[0][0])
                for comp in range(d):
                    for j, col in enumerate(vn[c]):
                        if not bnd[col]:
                            key = comp * Nv + int(col)
                            row[key] = row.get(key, 0.0) + B_t[c, li, comp, j]
                for j, col in enumerate(pn[c]):
                    key = d * Nv + int(col)
                    row[key] = row.get(key, 0.0) - c_p * Mp_t[c, li, j]
        out[n_i] = sum(abs(v) * abs(x[key]) for key, v in row.items())
    return out


def velocity_stencil(mesh, dofs):
    """Velocity DoFs (same component) of the cells around each velocity DoF in
    `dofs`: the entries a row of A reads."""
    d, k = mesh.dim, mesh.k
    Nv = mesh.n_vnode
    out = set()
    for g in dofs:
        comp, node = divmod(int(g), Nv)
        lat = mesh._unflat(np.array([node]), mesh.vel_dims)[0]
        cells = np.array(_cells_touching(mesh, lat, k))
        for n in mesh.cell_velocity_nodes(cells).ravel():
            out.add(comp * Nv + int(n))
    return np.array(sorted(out), dtype=np.int64)


def sample_diag_A(mesh, dofs, mu=1.0, gamma=0.0, rho=1.0):
    """diag(A) of the constrained velocity block at velocity DoFs `dofs`:
    1 on Dirichlet DoFs, else the sum over the cells around the node of the
    element matrix's diagonal entry."""
    k = mesh.k
    Nv = mesh.n_vnode
    bnd = mesh.velocity_boundary_nodes()
    mu_cell = mesh.mu(mu)
    out = np.zeros(len(dofs))
    for n_i, g in enumerate(dofs):
        comp, node = divmod(int(g), Nv)
        if bnd[node]:
            out[n_i] = 1.0
            continue
        lat = mesh._unflat(np.array([node]), mesh.vel_dims)[0]
        cells = np.array(_cells_touching(mesh, lat, k))
        A_t, _, _, _ = element_matrices(mesh, cells, mu_cell[cells], gamma, rho)
        vn = mesh.cell_velocity_nodes(cells)
        out[n_i] = sum(A_t[c, li, li] for c in range(len(cells)) for li in np.nonzero(vn[c] == node)[0])
    return out

