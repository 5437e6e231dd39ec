"""Pins of the oracle's discretisation (Section 2) against things other than
itself: the paper's printed DoF counts, hand-derived 1D element matrices,
exact symbolic integrals, quadrature exactness, symmetry and the discrete
divergence."""
import json
import os

import numpy as np
import pytest
import sympy

from oracle.fe import gll_points, gauss_rule, lagrange_values, lagrange_derivatives
from oracle.mesh import BoxMesh, make_hierarchy, taylor_hood_dof_count
from oracle.assemble import Assembled, element_matrices, CellData
import synth_inputs as si

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


@pytest.mark.parametrize("case", _gold("paper_dof_counts.json")["cases"])
def test_dof_counts_printed_in_paper(case):
    m = BoxMesh(case["dim"], (case["n"],) * case["dim"], case["k"])
    assert m.n_total == case["dofs"]
    assert taylor_hood_dof_count(case["dim"], case["n"], case["k"]) == case["dofs"]


def test_gll_points_closed_form():
    assert np.allclose(gll_points(3), [0.0, 0.5, 1.0], atol=1e-15)
    s = 1.0 / np.sqrt(5.0)
    assert np.allclose(gll_points(4), [0.0, (1 - s) / 2, (1 + s) / 2, 1.0], atol=1e-15)
    assert np.allclose(gll_points(2), [0.0, 1.0])


def test_gauss_rule_exactness():
    for nq in range(1, 7):
        x, w = gauss_rule(nq)
        for p in range(2 * nq):
            assert abs(np.dot(w, x ** p) - 1.0 / (p + 1)) < 1e-14


def test_lagrange_basis_is_nodal_and_derivative_matches_sympy():
    t = sympy.symbols("t")
    for npts in (2, 3, 4):
        z = gll_points(npts)
        V = lagrange_values(z, z)
        assert np.allclose(V, np.eye(npts), atol=1e-14)
        xs = np.linspace(0, 1, 7)
        G = lagrange_derivatives(z, xs)
        zs = [sympy.nsimplify(v) if npts < 4 else sympy.Float(v, 30) for v in z]
        for i in range(npts):
            li = sympy.Integer(1)
            for j in range(npts):
                if j != i:
                    li *= (t - zs[j]) / (zs[i] - zs[j])
            dli = sympy.lambdify(t, sympy.diff(li, t), "numpy")
            assert np.allclose(G[i], np.broadcast_to(dli(xs), xs.shape), atol=1e-12)


def test_cartesian_cell_matrices_are_tensor_products_of_textbook_1d_matrices():
    g = _gold("element_matrices_1d.json")
    hx, hy = 0.3, 0.7
    K1 = lambda h: np.array(g["q2_stiffness_times_3h"]) / (3 * h)
    M1 = lambda h: np.array(g["q2_mass_times_30_over_h"]) * h / 30
    Mq1 = lambda h: np.array(g["q1_mass_times_6_over_h"]) * h / 6
    G12 = np.array(g["q1_q2_derivative_times_6"]) / 6.0
    N12 = lambda h: np.array(g["q1_q2_mass_times_6_over_h"]) * h / 6
    mesh = BoxMesh(2, (1, 1), 2, lo=[0, 0], hi=[hx, hy])
    mu, gamma, rho = 1.7, 3.0, 0.9
    A, B, Mp, Mv = element_matrices(mesh, np.array([0]), np.array([mu]), gamma, rho)
    # lexicographic x-fastest local order: index = ix + 3 iy  -> kron(Y, X)
    A_ref = mu * (np.kron(M1(hy), K1(hx)) + np.kron(K1(hy), M1(hx))) + gamma * rho * np.kron(M1(hy), M1(hx))
    assert np.allclose(A[0], A_ref, rtol=1e-13, atol=1e-14)
    assert np.allclose(Mp[0], np.kron(Mq1(hy), Mq1(hx)), rtol=1e-13, atol=1e-15)
    Bx_ref = -np.kron(N12(hy), G12)
    By_ref = -np.kron(G12, N12(hx))
    assert np.allclose(B[0, :, 0, :], Bx_ref, rtol=1e-13, atol=1e-15)
    assert np.allclose(B[0, :, 1, :], By_ref, rtol=1e-13, atol=1e-15)
    # 3D: a(.,.) is a Kronecker sum over directions
    mesh3 = BoxMesh(3, (1, 1, 1), 2, lo=[0, 0, 0], hi=[hx, hy, 0.5])
    A3, B3, Mp3, _ = element_matrices(mesh3, np.array([0]), np.array([mu]), gamma, rho)
    hz = 0.5
    kr = lambda a, b, c: np.kron(a, np.kron(b, c))
    A3_ref = mu * (kr(M1(hz), M1(hy), K1(hx)) + kr(M1(hz), K1(hy), M1(hx)) + kr(K1(hz), M1(hy), M1(hx))) \
        + gamma * rho * kr(M1(hz), M1(hy), M1(hx))
    assert np.allclose(A3[0], A3_ref, rtol=1e-13, atol=1e-14)
    assert np.allclose(B3[0, :, 2, :], -kr(G12, N12(hy), N12(hx)), rtol=1e-13, atol=1e-15)


def _sympy_cell_forms(verts, k, mu, gr):
    """Exact integrals of a and b over a parallelogram cell via sympy, for
    test functions in the discrete spaces of an affine cell (total degree 2
    for velocity, 1 for pressure): u = x^2 + x y - y, v = x y - y^2 + x,
    q = 1 + 2x - y."""
    X, Y, s, t = sympy.symbols("X Y s t")
    v0, v1, v2, _ = [sympy.Matrix(v) for v in verts]
    xy = v0 + (v1 - v0) * s + (v2 - v0) * t          # affine map
    J = xy.jacobian([s, t])
    detJ = sympy.simplify(J.det())
    u = X ** 2 + X * Y - Y
    v = X * Y - Y ** 2 + X
    q = 1 + 2 * X - Y
    sub = {X: xy[0], Y: xy[1]}
    grad = lambda f: [sympy.diff(f, X), sympy.diff(f, Y)]
    a_int = (mu * (grad(u)[0] * grad(v)[0] + grad(u)[1] * grad(v)[1]) + gr * u * v).subs(sub) * detJ
    b_int = (-q * (grad(u)[0])).subs(sub) * detJ       # -int q d(u)/dx  (u in component x)
    a = sympy.integrate(sympy.expand(a_int), (s, 0, 1), (t, 0, 1))
    b = sympy.integrate(sympy.expand(b_int), (s, 0, 1), (t, 0, 1))
    return float(a), float(b), (u, v, q, X, Y)


def test_affine_cell_bilinear_forms_match_exact_symbolic_integrals():
    verts = [(0.1, 0.2), (0.9, 0.3), (0.3, 1.1), (1.1, 1.2)]     # parallelogram
    mesh = BoxMesh(2, (1, 1), 2, vertices=np.array(verts))
    mu, gr = 1.3, 2.5
    A, B, Mp, _ = element_matrices(mesh, np.array([0]), np.array([mu]), gr, 1.0)
    a_ex, b_ex, (u, v, q, X, Y) = _sympy_cell_forms(verts, 2, mu, gr)
    # nodal coefficient vectors: the nodes of the cell are the mapped lattice
    z = gll_points(3)
    zp = gll_points(2)
    V = np.array(verts)

    def node_xy(zz):
        pts = []
        for j in range(len(zz)):
            for i in range(len(zz)):
                s_, t_ = zz[i], zz[j]
                pts.append(V[0] + (V[1] - V[0]) * s_ + (V[2] - V[0]) * t_)
        return np.array(pts)
    fu = sympy.lambdify((X, Y), u)
    fv = sympy.lambdify((X, Y), v)
    fq = sympy.lambdify((X, Y), q)
    pv, pp = node_xy(z), node_xy(zp)
    cu = fu(pv[:, 0], pv[:, 1])
    cv = fv(pv[:, 0], pv[:, 1])
    cq = fq(pp[:, 0], pp[:, 1])
    assert abs(cv @ A[0] @ cu - a_ex) < 1e-12 * max(1, abs(a_ex))
    assert abs(cq @ B[0, :, 0, :] @ cu - b_ex) < 1e-12 * max(1, abs(b_ex))


def test_gauss_k_plus_1_is_exact_on_affine_cells_3d():
    # a parallelepiped: affine map, so k+1 Gauss points integrate exactly
    V = []
    e1, e2, e3 = np.array([0.8, 0.1, 0.0]), np.array([0.2, 0.9, 0.1]), np.array([0.1, -0.1, 0.7])
    for c in range(2):
        for b in range(2):
            for a in range(2):
                V.append(a * e1 + b * e2 + c * e3)
    mesh = BoxMesh(3, (1, 1, 1), 2, vertices=np.array(V))
    cd_lo = CellData(mesh, np.array([0]))
    cd_hi = CellData(mesh, np.array([0]), nq_1d=7)
    st = lambda cd: np.einsum("ciqa,cjqa,cq->cij", cd.grad, cd.grad, cd.JxW)
    bb = lambda cd: np.einsum("iq,cjqa,cq->ciaj", cd.psi, cd.grad, cd.JxW)
    assert np.allclose(st(cd_lo), st(cd_hi), rtol=1e-12, atol=1e-13)
    assert np.allclose(bb(cd_lo), bb(cd_hi), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("dim,k,n", [(2, 2, 4), (2, 3, 3), (3, 2, 2)])
def test_K_symmetric_and_Bt_one_zero(dim, k, n):
    rng = np.random.default_rng(0)
    verts = None
    if dim == 2:
        verts = si.perturbed_box_vertices(n, dim=2, amplitude=0.15, seed=11)
    mesh = BoxMesh(dim, (n,) * dim, k, vertices=verts)
    asm = Assembled(mesh, mu=1.3, gamma=10.0, rho=0.7, c_p=0.1)
    K = asm.K
    x, y = rng.standard_normal(K.shape[0]), rng.standard_normal(K.shape[0])
    assert abs(x @ (K @ y) - y @ (K @ x)) < 1e-13 * np.linalg.norm(x) * np.linalg.norm(y) * abs(K).max()
    # B^T 1 = 0 (unconstrained too): int div v = 0 for v vanishing on the boundary,
    # and pointwise sum of pressure basis = 1 -> column sums of B vanish for interior velocity nodes
    ones = np.ones(mesh.n_pnode)
    assert np.max(np.abs(asm.B.T @ ones)) < 1e-13
    # the constant pressure is in the kernel of K (with c_p = 0)
    asm0 = Assembled(mesh, mu=1.3, gamma=10.0, rho=0.7, c_p=0.0)
    e = np.concatenate([np.zeros(asm0.A.shape[0]), ones])
    assert np.max(np.abs(asm0.K @ e)) < 1e-13


def test_discrete_divergence_of_interpolated_divfree_field_converges():
    errs = []
    for n in (4, 8, 16):
        mesh = BoxMesh(2, (n, n), 2)
        asm = Assembled(mesh)
        X = mesh.velocity_node_coordinates()
        u = si.manufactured_u(X).T.ravel()
        r = asm.B @ u
        # scale by the pressure mass to get an L2-like norm of the discrete divergence
        Minv = 1.0 / asm.Mp.diagonal()
        errs.append(np.sqrt(r @ (Minv * r)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


def test_dirichlet_rows_are_identity():
    mesh = BoxMesh(2, (3, 3), 2)
    asm = Assembled(mesh)
    c = asm.constrained
    K = asm.K.tocsr()
    for i in c[:20]:
        row = K.getrow(i).toarray().ravel()
        assert row[i] == 1.0 and np.count_nonzero(row) == 1
        col = K.getcol(i).toarray().ravel()
        assert np.count_nonzero(col) == 1


def test_hierarchy_mu_averaging_and_vertex_subsampling():
    n_c, L = 2, 3
    nf = n_c * 2 ** (L - 1)
    V = si.perturbed_box_vertices(nf, dim=3, amplitude=0.2, seed=4)
    mu = si.fourier_log_viscosity(nf, dim=3, seed=5)
    ms = make_hierarchy(3, (n_c,) * 3, L, 3, fine_vertices=V, fine_mu=mu)
    assert ms[-1].mu_cell.shape == (nf ** 3,)
    assert np.isclose(ms[0].mu_cell.mean(), mu.mean())
    assert np.allclose(ms[-1].vertices, V)
    assert np.allclose(mu.min(), 1.0) and np.allclose(mu.max(), 100.0)
    # coarse vertex (1,1,1) of level 0 is fine vertex (4,4,4)
    i_c = 1 + 3 * (1 + 3 * 1)
    i_f = 4 + (nf + 1) * (4 + (nf + 1) * 4)
    assert np.allclose(ms[0].vertices[i_c], V[i_f])
