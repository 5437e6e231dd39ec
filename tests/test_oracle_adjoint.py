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


@pytest.mark.parametrize("c_p", [0.0, 0.5])
def test_pressure_objective_gradient_matches_central_differences(c_p):
    """J = ||x - t||^2 over velocity and pressure of the returned solution:
    for C = 0 the pressure is the mean-free one and the adjoint right-hand
    side takes the transpose of that normalisation; for C = c_p M_p, c_p > 0,
    the solve is the plain one.  Central differences of J in random
    directions of (log mu, f)."""
    from oracle.adjoint import state_solve, normalisation_adjoint
    dim, n, k = 2, (4, 3), 2
    V, logmu, f, _ = _problem(dim, n, k, seed=51)

    def J(lm, ff):
        mesh = BoxMesh(dim, n, k, vertices=V, mu_cell=np.exp(lm))
        asm = Assembled(mesh, gamma=2.0, rho=1.0, c_p=c_p)
        x = state_solve(asm, rhs_from_force(asm, ff))
        return x, asm

    x, asm = J(logmu, f)
    t = si.uniform(len(x), 52)
    J0 = float((x - t) @ (x - t))
    lam = state_solve(asm, normalisation_adjoint(asm, 2.0 * (x - t)))
    g_mu, g_f = gradients(asm, x, lam)
    rng = np.random.default_rng(8)
    h = 1e-6
    for _ in range(3):
        dmu = rng.standard_normal(len(logmu))
        df = rng.standard_normal(len(f))
        xp = J(logmu + h * dmu, f + h * df)[0]
        xm = J(logmu - h * dmu, f - h * df)[0]
        fd = (float((xp - t) @ (xp - t)) - float((xm - t) @ (xm - t))) / (2 * h)
        an = g_mu @ dmu + g_f @ df
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3 * J0), (fd, an)
    if c_p == 0.0:
        # the bordered solve applies that transpose by itself: its multiplier
        # s takes up the inconsistent part, K lam = g - m s with
        # s = (1.g_p)/(1.m), so both right-hand sides give the same lam_u;
        # the projected one is also consistent (orthogonal to (0, 1))
        g = 2.0 * (x - t)
        gp = normalisation_adjoint(asm, g)
        nu = asm.A.shape[0]
        assert abs(gp[nu:].sum()) <= 1e-13 * np.abs(g[nu:]).sum()
        lam_raw = state_solve(asm, g)
        assert np.allclose(lam_raw[:nu], lam[:nu], rtol=1e-10, atol=1e-12 * np.abs(lam[:nu]).max())
