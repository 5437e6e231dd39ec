"""Pins of the oracle's lifting of non-homogeneous Dirichlet data (Sec. 2):
a Stokes / generalized Stokes solution that lies in the discrete spaces
(quadratic velocity, linear pressure) with non-zero boundary values is
reproduced exactly from its boundary values and its force, and the driven
cavity's boundary data are compatible (zero net flux)."""
import numpy as np
import pytest

from oracle.mesh import BoxMesh
from oracle.assemble import Assembled, rhs_closed_form
from oracle.adjoint import bordered_solve
from oracle.dirichlet import lift, insert, lid_driven_cavity, extend_by_zero


def _exact(dim, mu, gr):
    """u with each component quadratic in the other coordinates (div u = 0),
    p linear with zero mean on the unit box, f = -mu Lap u + gr u + grad p."""
    def u(X):
        if dim == 2:
            return np.stack([X[:, 1] ** 2, X[:, 0] ** 2], axis=1)
        return np.stack([X[:, 1] ** 2 + X[:, 2] ** 2, X[:, 0] ** 2 + X[:, 2] ** 2, X[:, 0] ** 2 + X[:, 1] ** 2], axis=1)

    def p(X):
        return X.sum(axis=1) - 0.5 * dim

    lap = 2.0 * (dim - 1)     # Laplacian of every component

    def f(X):
        return -mu * lap + gr * u(X) + 1.0

    return u, p, f


def _pressure_coords(mesh):
    # uniform box on [0, 1]^d: the Q_{k-1} GLL nodes are equally spaced for k <= 3
    idx = mesh._unflat(np.arange(mesh.n_pnode), mesh.p_dims)
    return idx / np.array([(mesh.k - 1) * v for v in mesh.n], dtype=np.float64)


@pytest.mark.parametrize("dim,n,k,gamma", [(2, (3, 4), 2, 0.0), (2, (3, 2), 3, 5.0), (3, (2, 3, 2), 2, 2.0)])
def test_lifting_reproduces_a_solution_in_the_discrete_space(dim, n, k, gamma):
    mu = 1.7
    mesh = BoxMesh(dim, n, k)
    asm = Assembled(mesh, mu=mu, gamma=gamma, rho=1.0)
    u, p, f = _exact(dim, mu, gamma)
    X = mesh.velocity_node_coordinates()
    u_nodal = u(X).T.ravel()
    b = rhs_closed_form(mesh, f)
    x = insert(asm, bordered_solve(asm, lift(asm, b, u_nodal)), u_nodal)
    nu = asm.A.shape[0]
    assert np.max(np.abs(x[:nu] - u_nodal)) < 1e-10
    assert np.max(np.abs(x[nu:] - p(_pressure_coords(mesh)))) < 1e-10


def test_lifting_without_the_lift_term_fails_the_pin():
    # the same problem solved as if u_D were 0 is far from the exact solution
    mesh = BoxMesh(2, (3, 4), 2)
    asm = Assembled(mesh, mu=1.0)
    u, p, f = _exact(2, 1.0, 0.0)
    u_nodal = u(mesh.velocity_node_coordinates()).T.ravel()
    x = insert(asm, bordered_solve(asm, rhs_closed_form(mesh, f)), u_nodal)
    assert np.max(np.abs(x[:asm.A.shape[0]] - u_nodal)) > 1e-2


def test_lift_with_zero_data_only_clears_dirichlet_rows():
    mesh = BoxMesh(2, (3, 3), 2)
    asm = Assembled(mesh, gamma=1.0)
    b = np.random.default_rng(0).standard_normal(asm.K.shape[0])
    out = lift(asm, b, np.zeros(asm.A.shape[0]))
    ref = b.copy()
    ref[:asm.A.shape[0]] *= asm.free_u
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("dim,n", [(2, (4, 4)), (3, (2, 2, 2))])
def test_cavity_data_tangential_and_flux_free(dim, n):
    mesh = BoxMesh(dim, n, 2)
    asm = Assembled(mesh)
    ud = lid_driven_cavity(mesh)
    ut = extend_by_zero(asm, ud)
    assert np.array_equal(ut, ud)                   # only boundary nodes carry data
    assert np.all(ud.reshape(dim, -1)[1:] == 0)     # tangential: along x only
    # int div u~ = 0: the pressure rows of the lifted system sum to zero
    assert abs(np.sum(asm.B_unconstrained @ ut)) < 1e-13
    assert np.count_nonzero(ud) == np.prod([2 * v - 1 for v in n[:-1]])
