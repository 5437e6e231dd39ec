"""Box-mesh hierarchy and Taylor-Hood DoF numbering (oracle; test infrastructure only).

Section 3.1: meshes T_0 ... T_L, T_l obtained from T_{l-1} by uniform
refinement, so cells per direction double from level to level.  Section 2:
each cell is the image of (0,1)^d under a bi-/trilinear map T_tau given by its
2^d vertices, and the nodes are the tensor-product lattice mapped by T_tau.

Numbering (the vector layout shared with the library's interface):
  * velocity lattice per component: (k n_x + 1) x (k n_y + 1) [x (k n_z + 1)]
    nodes, index ix + Lx*(iy + Ly*iz) (x fastest);
  * pressure lattice: ((k-1) n_x + 1) x ... with the same ordering;
  * global vector [u_1 | u_2 | (u_3) | p].
All velocity nodes on the boundary of the box carry the homogeneous Dirichlet
condition of Eqs. (1)-(2).

Perturbed hierarchies (a reading: the paper's own meshes are adapted to the
geometry during refinement and so are not nested either): level l takes the
finest-level vertex at the same lattice point; the per-cell viscosity of a
coarse cell is the mean over its 2^d children.
"""
import numpy as np


class BoxMesh:
    def __init__(self, dim, n, k, lo=None, hi=None, vertices=None, mu_cell=None):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if k < 2:
            raise ValueError("Taylor-Hood needs k >= 2")
        self.dim = dim
        self.n = tuple(int(v) for v in (list(n) + [1, 1])[:dim])
        self.k = k
        self.lo = np.zeros(dim) if lo is None else np.asarray(lo, dtype=np.float64)[:dim]
        self.hi = np.ones(dim) if hi is None else np.asarray(hi, dtype=np.float64)[:dim]
        self.nvert = tuple(v + 1 for v in self.n)
        if vertices is None:
            axes = [np.linspace(self.lo[a], self.hi[a], self.nvert[a]) for a in range(dim)]
            grids = np.meshgrid(*axes, indexing="ij")
            # flatten with x fastest
            vertices = np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids], axis=1)
            self.cartesian = True
        else:
            self.cartesian = False
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, dim)
        assert self.vertices.shape[0] == int(np.prod(self.nvert))
        self.ncell = int(np.prod(self.n))
        self.mu_cell = None if mu_cell is None else np.asarray(mu_cell, dtype=np.float64).reshape(self.ncell)
        self.vel_dims = tuple(k * v + 1 for v in self.n)
        self.p_dims = tuple((k - 1) * v + 1 for v in self.n)
        self.n_vnode = int(np.prod(self.vel_dims))
        self.n_pnode = int(np.prod(self.p_dims))
        self.n_u = dim * self.n_vnode
        self.n_p = self.n_pnode
        self.n_total = self.n_u + self.n_p

    # ---- lattice helpers -------------------------------------------------
    @staticmethod
    def _flat(idx, dims):
        out = np.zeros(idx.shape[0], dtype=np.int64)
        stride = 1
        for a in range(len(dims)):
            out += idx[:, a].astype(np.int64) * stride
            stride *= dims[a]
        return out

    @staticmethod
    def _unflat(flat, dims):
        flat = np.asarray(flat, dtype=np.int64)
        out = np.zeros((flat.shape[0], len(dims)), dtype=np.int64)
        for a in range(len(dims)):
            out[:, a] = flat % dims[a]
            flat = flat // dims[a]
        return out

    def cell_index(self, cells):
        return self._unflat(cells, self.n)

    def cell_vertex_ids(self, cells):
        c = self.cell_index(cells)
        corners = np.indices((2,) * self.dim).reshape(self.dim, -1)[::-1].T
        out = np.zeros((len(c), len(corners)), dtype=np.int64)
        for j, off in enumerate(corners):
            out[:, j] = self._flat(c + off[None, :], self.nvert)
        return out

    def _cell_lattice_dofs(self, cells, npts, dims):
        c = self.cell_index(cells)
        loc = np.indices((npts,) * self.dim).reshape(self.dim, -1)[::-1].T
        out = np.zeros((len(c), len(loc)), dtype=np.int64)
        for j, off in enumerate(loc):
            out[:, j] = self._flat(c * (npts - 1) + off[None, :], dims)
        return out

    def cell_velocity_nodes(self, cells):
        return self._cell_lattice_dofs(cells, self.k + 1, self.vel_dims)

    def cell_pressure_nodes(self, cells):
        return self._cell_lattice_dofs(cells, self.k, self.p_dims)

    def velocity_boundary_nodes(self):
        """Boolean mask over velocity lattice nodes lying on the box boundary."""
        idx = self._unflat(np.arange(self.n_vnode), self.vel_dims)
        mask = np.zeros(self.n_vnode, dtype=bool)
        for a in range(self.dim):
            mask |= (idx[:, a] == 0) | (idx[:, a] == self.vel_dims[a] - 1)
        return mask

    def constrained_dofs(self):
        """Global indices (into [u_1|...|u_d|p]) of Dirichlet velocity DoFs."""
        nodes = np.nonzero(self.velocity_boundary_nodes())[0]
        return np.concatenate([nodes + c * self.n_vnode for c in range(self.dim)])

    def mu(self, default):
        if self.mu_cell is not None:
            return self.mu_cell
        return np.full(self.ncell, float(default))

    # ---- geometry --------------------------------------------------------
    def map_points(self, cells, xi):
        """Physical coordinates T_tau(xi) for reference points xi[npt, dim]."""
        X = self.vertices[self.cell_vertex_ids(cells)]          # (nc, 2^d, dim)
        N = multilinear_shape(xi, self.dim)                       # (npt, 2^d)
        return np.einsum("pv,cva->cpa", N, X)

    def velocity_node_coordinates(self):
        """Physical coordinates of every velocity lattice node (each node is
        mapped from one cell that contains it; the map is continuous)."""
        from .fe import gll_points
        k, d = self.k, self.dim
        z = gll_points(k + 1)
        idx = self._unflat(np.arange(self.n_vnode), self.vel_dims)
        cell = np.minimum(idx // k, np.array(self.n) - 1)
        loc = idx - cell * k
        xi = z[loc]                                               # (nn, d)
        cells = self._flat(cell, self.n)
        X = self.vertices[self.cell_vertex_ids(cells)]
        out = np.zeros((self.n_vnode, d))
        for a in range(d):
            Nv = np.ones((self.n_vnode, 2 ** d))
            corners = np.indices((2,) * d).reshape(d, -1)[::-1].T
            for j, off in enumerate(corners):
                for b in range(d):
                    Nv[:, j] *= xi[:, b] if off[b] else (1.0 - xi[:, b])
            out[:, a] = np.einsum("nv,nv->n", Nv, X[:, :, a])
        return out


def multilinear_shape(xi, dim):
    """Values N_v(xi) of the 2^d multilinear vertex functions (x fastest)."""
    xi = np.atleast_2d(xi)
    corners = np.indices((2,) * dim).reshape(dim, -1)[::-1].T
    N = np.ones((xi.shape[0], len(corners)))
    for j, off in enumerate(corners):
        for b in range(dim):
            N[:, j] *= xi[:, b] if off[b] else (1.0 - xi[:, b])
    return N


def multilinear_shape_grad(xi, dim):
    """Reference gradients dN_v/dxi_b, shape (npt, 2^d, dim)."""
    xi = np.atleast_2d(xi)
    corners = np.indices((2,) * dim).reshape(dim, -1)[::-1].T
    G = np.ones((xi.shape[0], len(corners), dim))
    for j, off in enumerate(corners):
        for b in range(dim):
            for c in range(dim):
                if c == b:
                    G[:, j, b] *= 1.0 if off[c] else -1.0
                else:
                    G[:, j, b] *= xi[:, c] if off[c] else (1.0 - xi[:, c])
    return G


def make_hierarchy(dim, n_coarse, n_levels, k, lo=None, hi=None,
                   fine_vertices=None, fine_mu=None):
    """Meshes for levels 0 (coarsest) .. n_levels-1 (finest)."""
    n_coarse = tuple(int(v) for v in (list(n_coarse) + [n_coarse[0]] * 3)[:dim])
    L = n_levels - 1
    n_fine = tuple(v * 2 ** L for v in n_coarse)
    meshes = []
    mu_lvl = None if fine_mu is None else np.asarray(fine_mu, dtype=np.float64)
    mus = [None] * n_levels
    if mu_lvl is not None:
        mus[L] = mu_lvl.reshape(n_fine[::-1])       # (nz, ny, nx) view, x fastest
        for l in range(L - 1, -1, -1):
            m = mus[l + 1]
            if dim == 2:
                m = 0.25 * (m[0::2, 0::2] + m[0::2, 1::2] + m[1::2, 0::2] + m[1::2, 1::2])
            else:
                m = 0.125 * sum(m[a::2, b::2, c::2] for a in (0, 1) for b in (0, 1) for c in (0, 1))
            mus[l] = m
    for l in range(n_levels):
        n_l = tuple(v * 2 ** l for v in n_coarse)
        verts = None
        if fine_vertices is not None:
            s = 2 ** (L - l)
            fv = np.asarray(fine_vertices, dtype=np.float64).reshape(tuple(v + 1 for v in n_fine[::-1]) + (dim,))
            if dim == 2:
                verts = fv[::s, ::s].reshape(-1, dim)
            else:
                verts = fv[::s, ::s, ::s].reshape(-1, dim)
        mu_l = None if mus[l] is None else mus[l].reshape(-1)
        meshes.append(BoxMesh(dim, n_l, k, lo, hi, vertices=verts, mu_cell=mu_l))
    return meshes


def taylor_hood_dof_count(dim, n, k):
    """N = d (k n + 1)^d + ((k-1) n + 1)^d on an n^d box mesh."""
    return dim * (k * n + 1) ** dim + ((k - 1) * n + 1) ** dim
