"""Pins of the oracle's deformation-rate form a_eps(u,v) = int mu eps(u):eps(v)
+ gamma rho u.v (Sec. 2): rigid motions span its kernel, integrals of
polynomial fields against their closed forms, a divergence-free quadratic
solution reproduced from its boundary values, and adjoint gradients against
central differences."""
import numpy as np
import pytest

import synth_inputs as si
from oracle.mesh import BoxMesh
from oracle.assemble import Assembled, rhs_closed_form
from oracle.adjoint import bordered_solve, rhs_from_force, velocity_objective, gradients
from oracle.dirichlet import lift, insert


def _fields(mesh, funcs):
    X = mesh.velocity_node_coordinates()
    return np.concatenate([f(X) for f in funcs])


@pytest.mark.parametrize("dim,n", [(2, (3, 4)), (3, (2, 2, 3))])
def test_rigid_motions_span_the_kernel(dim, n):
    V = si.perturbed_box_vertices(n, dim=dim, amplitude=0.2, seed=5)
    mesh = BoxMesh(dim, n, 2, vertices=V, mu_cell=si.uniform(int(np.prod(n)), 6, 0.5, 2.0))
    sym = Assembled(mesh, form="sym").A_unconstrained
    grad = Assembled(mesh).A_unconstrained
    zero = lambda X: np.zeros(len(X))
    one = lambda X: np.ones(len(X))
    if dim == 2:
        motions = [[one, zero], [zero, one], [lambda X: -X[:, 1], lambda X: X[:, 0]]]
    else:
        x, y, z = (lambda X: X[:, 0]), (lambda X: X[:, 1]), (lambda X: X[:, 2])
        neg = lambda f: (lambda X: -f(X))
        motions = [[one, zero, zero], [zero, one, zero], [zero, zero, one],
                   [neg(y), x, zero], [zero, neg(z), y], [z, zero, neg(x)]]
    for m in motions:
        r = _fields(mesh, m)
        assert np.max(np.abs(sym @ r)) < 1e-12 * np.max(np.abs(sym.data))
    rot = _fields(mesh, motions[-1])
    assert np.max(np.abs(grad @ rot)) > 1e-3        # the gradient form does not vanish on rotations


# (u, v, int eps(u):eps(v)) on the unit box, mu = 1: quadratic fields, so their
# Q2 interpolants are exact
Z = lambda X: np.zeros(len(X))
CASES_2D = [
    ([Z, lambda X: X[:, 0] ** 2], [lambda X: X[:, 1] ** 2, Z], 0.5),          # eps_12 eps_12 coupling
    ([lambda X: X[:, 0] ** 2, Z], [lambda X: X[:, 0] * X[:, 1], Z], 0.5),     # eps_11
    ([lambda X: X[:, 1] ** 2, Z], [lambda X: X[:, 0] * X[:, 1], Z], 0.25),    # eps_12 within one component
]
CASES_3D = [
    ([Z, Z, lambda X: X[:, 0] ** 2], [lambda X: X[:, 2] ** 2, Z, Z], 0.5),
    ([Z, lambda X: X[:, 2] ** 2, Z], [Z, Z, lambda X: X[:, 1] ** 2], 0.5),
    ([lambda X: X[:, 0] * X[:, 1], Z, Z], [lambda X: X[:, 0] ** 2, Z, Z], 0.5),
]


@pytest.mark.parametrize("dim,case", [(2, c) for c in CASES_2D] + [(3, c) for c in CASES_3D])
def test_integrals_of_polynomial_fields(dim, case):
    u, v, ref = case
    mesh = BoxMesh(dim, (2,) * dim, 2)
    A = Assembled(mesh, form="sym").A_unconstrained
    val = _fields(mesh, v) @ (A @ _fields(mesh, u))
    assert abs(val - ref) < 1e-13


@pytest.mark.parametrize("dim,n,k", [(2, (3, 4), 2), (2, (3, 2), 3), (3, (2, 2, 2), 2)])
def test_quadratic_solution_reproduced(dim, n, k):
    """-div(mu eps(u)) + grad p = f: for div u = 0, div eps(u) = Lap u / 2."""
    mu, gr = 1.4, 3.0
    mesh = BoxMesh(dim, n, k)
    asm = Assembled(mesh, mu=mu, gamma=gr, rho=1.0, form="sym")
    if dim == 2:
        U = lambda X: np.stack([X[:, 1] ** 2, X[:, 0] ** 2], axis=1)
    else:
        U = lambda X: np.stack([X[:, 1] ** 2 + X[:, 2] ** 2, X[:, 0] ** 2 + X[:, 2] ** 2,
                                X[:, 0] ** 2 + X[:, 1] ** 2], axis=1)
    f = lambda X: -0.5 * mu * 2.0 * (dim - 1) + gr * U(X) + 1.0
    u_nodal = U(mesh.velocity_node_coordinates()).T.ravel()
    x = insert(asm, bordered_solve(asm, lift(asm, rhs_closed_form(mesh, f), u_nodal)), u_nodal)
    nu = asm.A.shape[0]
    idx = mesh._unflat(np.arange(mesh.n_pnode), mesh.p_dims)
    p = (idx / np.array([(k - 1) * v for v in n], dtype=np.float64)).sum(axis=1) - 0.5 * dim
    assert np.max(np.abs(x[:nu] - u_nodal)) < 1e-10
    assert np.max(np.abs(x[nu:] - p)) < 1e-10


def test_adjoint_gradient_central_differences_sym():
    dim, n, k = 2, (3, 3), 2
    V = si.perturbed_box_vertices(n, dim=dim, amplitude=0.2, seed=8)
    logmu = np.log(si.uniform(9, 9, 0.5, 3.0))
    f = si.uniform(2 * 49, 10)
    ut = si.uniform(2 * 49, 11)

    def J(lm, ff):
        asm = Assembled(BoxMesh(dim, n, k, vertices=V, mu_cell=np.exp(lm)), gamma=1.0, form="sym")
        x = bordered_solve(asm, rhs_from_force(asm, ff))
        val, g = velocity_objective(asm, x, ut)
        return val, g, x, asm

    J0, g, x, asm = J(logmu, f)
    g_mu, g_f = gradients(asm, x, bordered_solve(asm, g))
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(3):
        dm = rng.standard_normal(len(logmu))
        df = rng.standard_normal(len(f))
        fd = (J(logmu + h * dm, f + h * df)[0] - J(logmu - h * dm, f - h * df)[0]) / (2 * h)
        assert abs(fd - (g_mu @ dm + g_f @ df)) <= 1e-6 * max(abs(fd), 1e-3 * J0)
