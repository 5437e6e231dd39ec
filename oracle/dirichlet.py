"""Non-homogeneous Dirichlet data by lifting (oracle; test infrastructure only).

Section 2 prescribes u = u_D on the boundary; the constrained system K of
`assemble` is homogeneous there (identity rows, zero columns).  With u~ the
discrete field equal to u_D on the Dirichlet nodes and 0 at every other
node, the solution is u = u0 + u~ with u0 homogeneous on the boundary and

  K x0 = b - K_full u~   on the free velocity rows and the pressure rows,
  x0 = 0                 on the Dirichlet rows,

where K_full = [A_full B_full^T; B_full -C] is the operator before the
constraints (A_full, B_full keep their Dirichlet columns).  The pressure part
of K_full u~ is B_full u~.
"""
import numpy as np


def extend_by_zero(asm, u_d):
    """u~: the velocity vector equal to u_d on the Dirichlet nodes, 0 elsewhere."""
    ut = np.zeros(asm.A.shape[0])
    c = asm.mesh.constrained_dofs()
    ut[c] = np.asarray(u_d, dtype=np.float64)[c]
    return ut


def lift(asm, b, u_d):
    """Right-hand side of the homogeneous problem for the data u_d."""
    nu = asm.A.shape[0]
    ut = extend_by_zero(asm, u_d)
    out = np.array(b, dtype=np.float64, copy=True)
    out[:nu] -= asm.A_unconstrained @ ut
    out[:nu] *= asm.free_u
    out[nu:] -= asm.B_unconstrained @ ut
    return out


def insert(asm, x0, u_d):
    """x = x0 + u~ for x0 homogeneous on the boundary, i.e. x0 with its
    Dirichlet entries replaced by u_d."""
    x = np.array(x0, dtype=np.float64, copy=True)
    c = asm.mesh.constrained_dofs()
    x[c] = np.asarray(u_d, dtype=np.float64)[c]
    return x


def lid_driven_cavity(mesh, lid=1.0):
    """u_D of the driven cavity (Sec. 4): tangential velocity `lid` along x on
    the top face (y = 1 in 2D, z = 1 in 3D), 0 on the other faces.  Nodes on
    the edges of the top face belong to the fixed walls (u_D = 0 there)."""
    d = mesh.dim
    idx = mesh._unflat(np.arange(mesh.n_vnode), mesh.vel_dims)
    top = idx[:, d - 1] == mesh.vel_dims[d - 1] - 1
    inner = np.ones(mesh.n_vnode, dtype=bool)
    for a in range(d - 1):
        inner &= (idx[:, a] > 0) & (idx[:, a] < mesh.vel_dims[a] - 1)
    u = np.zeros((d, mesh.n_vnode))
    u[0, top & inner] = lid
    return u.ravel()
