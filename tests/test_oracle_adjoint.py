"""Pins of the oracle's adjoint-state gradients: central finite differences of
J(f, log mu) = ||u(f, mu) - u_target||^2 with direct solves on tiny meshes."""
import numpy as np
import pytest

import synth_inputs as si
from oracle.assemble import Assembled
from oracle.mesh import BoxMesh
from oracle.adjoint import bordered_solve, rhs_from_force, velocity_objective, gradients


def _problem(dim, n, k, seed):
    V = si.perturbed_box_vertices(n, dim=dim, amplitude=0.2, seed=seed)
    ncell = int(np.prod(n))
    logmu = np.log(si.uniform(ncell, seed + 1, 0.5, 3.0))
    mesh0 = BoxMesh(dim, n, k, vertices=V)
    f = si.uniform(mesh0.n_u, seed + 2)
    ut = si.uniform(mesh0.n_u, seed + 3)
    return V, logmu, f, ut


def _J(dim, n, k, V, logmu, f, ut, gamma=2.0):
    mesh = BoxMesh(dim, n, k, vertices=V, mu_cell=np.exp(logmu))
    asm = Assembled(mesh, gamma=gamma, rho=1.0)
    x = bordered_solve(asm, rhs_from_force(asm, f))
    J, g = velocity_objective(asm, x, ut)
    return J, g, x, asm


@pytest.mark.parametrize("dim,n,k", [(2, (4, 3), 2), (2, (3, 3), 3), (3, (2, 2, 2), 2)])
def test_adjoint_gradient_matches_central_differences(dim, n, k):
    V, logmu, f, ut = _problem(dim, n, k, seed=31)
    J0, g, x, asm = _J(dim, n, k, V, logmu, f, ut)
    lam = bordered_solve(asm, g)
    g_mu, g_f = gradients(asm, x, lam)
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(3):
        dmu = rng.standard_normal(len(logmu))
        Jp = _J(dim, n, k, V, logmu + h * dmu, f, ut)[0]
        Jm = _J(dim, n, k, V, logmu - h * dmu, f, ut)[0]
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g_mu @ dmu) <= 1e-6 * max(abs(fd), 1e-3 * J0)
        df = rng.standard_normal(len(f))
        Jp = _J(dim, n, k, V, logmu, f + h * df, ut)[0]
        Jm = _J(dim, n, k, V, logmu, f - h * df, ut)[0]
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g_f @ df) <= 1e-6 * max(abs(fd), 1e-3 * J0)


def test_gradient_of_viscosity_vanishes_for_zero_adjoint():
    V, logmu, f, ut = _problem(2, (3, 3), 2, seed=5)
    _, g, x, asm = _J(2, (3, 3), 2, V, logmu, f, ut)
    g_mu, g_f = gradients(asm, x, np.zeros_like(x))
    assert np.all(g_mu == 0) and np.all(g_f == 0)
