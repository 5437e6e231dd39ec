"""Pins of the oracle's smoother, transfers, coarse solve and outer loops
(Sections 3.1-3.3, 4.1) against closed forms, dense linear algebra and the
qualitative behaviour the paper reports."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.mesh import BoxMesh, make_hierarchy
from oracle.assemble import Assembled, rhs_closed_form, CellData
from oracle.smoother import (LevelSmoother, chebyshev_apply, scaling_constant,
                             chebyshev_first_kind, splitmix64_u64, lanczos_max, schur_diagonal)
from oracle.transfer import prolongation, _field_prolongation
from oracle.mg import Multigrid, pressure_mean_free
from oracle.krylov import fgmres, stationary, rate_q, time_to_reduce
from oracle.rows import sample_Kx
import synth_inputs as si

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# --------------------------------------------------------------------------
# Chebyshev-Jacobi (Sec. 3.3.1, Lemma 1, Algorithm 2)
# --------------------------------------------------------------------------
def test_scaling_constants_closed_form():
    g = _gold("chebyshev_constants.json")
    for k in range(4):
        assert chebyshev_first_kind(k + 1, 3.0) == g["C_at_3"][k]
        num, den = g["sigma_num_den"][k]
        assert abs(scaling_constant(k) - num / den) < 1e-16


def test_eta0_smoothing_factor_formula():
    g = _gold("chebyshev_constants.json")
    for m, ref in zip(range(1, 6), g["eta0_m1_to_m5"]):
        assert 2.0 ** (-m) * math.comb(m, (m + 1) // 2) == ref


def _cheb_T_closed(n, x):
    """C_n by its trigonometric/hyperbolic definition (independent of numpy's series)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(n * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** n * np.cosh(n * np.arccosh(np.abs(xo)))
    return out


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_chebyshev_recurrence_reproduces_s_k_on_a_diagonal_matrix(k):
    beta = 2.3
    alpha = beta / 2
    lam = np.linspace(0.05, beta, 57)   # away from 0, where (1 - T)/lam cancels
    out = chebyshev_apply(lambda v: lam * v, np.ones_like(lam), np.ones_like(lam), k, beta)
    T = _cheb_T_closed(k + 1, (beta + alpha - 2 * lam) / (beta - alpha)) / \
        _cheb_T_closed(k + 1, np.array([(beta + alpha) / (beta - alpha)]))[0]
    s_k = (1.0 - T) / lam
    assert np.allclose(out, s_k, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_lemma1_bounds(k):
    beta = 1.0
    lam = np.linspace(1e-6, beta, 200001)
    s = chebyshev_apply(lambda v: lam * v, np.ones_like(lam), np.ones_like(lam), k, beta)
    C = chebyshev_first_kind(k + 1, 3.0)
    assert abs(np.max(lam * s) - (1 + 1 / C)) < 1e-9
    assert np.min(s) >= (1 - 1 / C) / beta - 1e-12


def test_damped_jacobi_case():
    # k = 0: omega = 2/(alpha+beta); sigma = 3/4 -> A_hat^-1 = D^-1 / beta
    D = np.array([2.0, 3.0, 5.0])
    r = np.array([1.0, -2.0, 0.5])
    beta = 1.7
    out = scaling_constant(0) * chebyshev_apply(None, 1 / D, r, 0, beta)
    assert np.allclose(out, r / D / beta, rtol=1e-15)


@pytest.mark.parametrize("kA", [0, 1, 3])
def test_exact_schur_diagonal_from_the_spectral_form(kA):
    """D_S~ = diag(B A_hat^-1 B^T) (+ diag C) of Sec. 3.3.1, with A_hat^-1 =
    sigma D^-1/2 Q s_k(Lambda) Q^T D^-1/2 built from the eigen-decomposition of
    D^-1/2 A D^-1/2 and the closed-form residual polynomial of the Chebyshev
    iteration, against the oracle's probing with unit vectors."""
    mesh = BoxMesh(2, (3, 4), 2, vertices=si.perturbed_box_vertices((3, 4), dim=2, amplitude=0.15, seed=3),
                   mu_cell=si.uniform(12, 4, 0.5, 2.0))
    asm = Assembled(mesh, gamma=2.0, rho=1.0, c_p=0.3)
    sm = LevelSmoother(asm, k_A=kA, k_S=1, schur="exact")
    A = asm.A.toarray()
    dh = 1.0 / np.sqrt(np.diag(A))
    lam, Q = np.linalg.eigh(dh[:, None] * A * dh[None, :])
    beta = sm.beta_A
    alpha = beta / 2
    T = _cheb_T_closed(kA + 1, (beta + alpha - 2 * lam) / (beta - alpha)) / \
        _cheb_T_closed(kA + 1, np.array([(beta + alpha) / (beta - alpha)]))[0]
    Ahat_inv = scaling_constant(kA) * (dh[:, None] * (Q * ((1.0 - T) / lam)) @ Q.T * dh[None, :])
    B = asm.B.toarray()
    ref = np.einsum("ij,jk,ik->i", B, Ahat_inv, B) + 0.3 * asm.Mp.diagonal()
    assert np.allclose(sm.D_S, ref, rtol=1e-10, atol=0)
    if kA == 0:
        # damped Jacobi: A_hat^-1 = D_A^-1 / beta_A, so D_S~ = D~_S_d / beta_A on the B part
        d = schur_diagonal(asm, "d") - 0.3 * asm.Mp.diagonal()
        assert np.allclose(sm.D_S - 0.3 * asm.Mp.diagonal(), d / beta, rtol=1e-12)


def test_splitmix64_published_vector():
    # published SplitMix64 reference outputs for seed 0
    assert [hex(z) for z in splitmix64_u64(0, 3)] == ["0xe220a8397b1dcdaf", "0x6e789e6aa1b965f4", "0x6c45d188009454f"]


def test_lanczos_close_to_dense_lambda_max():
    mesh = BoxMesh(2, (8, 8), 2)
    asm = Assembled(mesh, gamma=5.0)
    S = LevelSmoother(asm, 2, 1)
    A = asm.A.toarray()
    D = np.diag(A)
    lam = np.max(np.linalg.eigvalsh(A / np.sqrt(D)[:, None] / np.sqrt(D)[None, :]))
    assert abs(S.beta_A / 1.02 - lam) < 0.01 * lam
    assert S.beta_A >= lam
    # Schur: dense S~ = B A_hat^-1 B^T
    n_p = asm.B.shape[0]
    Sd = np.column_stack([S.S_tilde(np.eye(n_p)[:, i]) for i in range(n_p)])
    DS = S.D_S
    lamS = np.max(np.linalg.eigvalsh(Sd / np.sqrt(DS)[:, None] / np.sqrt(DS)[None, :]))
    assert abs(S.beta_S / 1.02 - lamS) < 0.01 * lamS


def _dense_Ahat_inv(S):
    n = S.nu
    return np.column_stack([S.Ainv(np.eye(n)[:, i]) for i in range(n)])


@pytest.mark.parametrize("kA,kS,schur", [(1, 1, "d"), (2, 1, "p"), (0, 2, "loc"), (3, 3, "d")])
def test_smoother_step_equals_compact_form_and_spectral_inequalities(kA, kS, schur):
    mesh = BoxMesh(2, (3, 3), 2)
    asm = Assembled(mesh, mu=1.0, gamma=2.0)
    S = LevelSmoother(asm, kA, kS, schur)
    nu = S.nu
    A = asm.A.toarray()
    B = asm.B.toarray()
    K = asm.K.toarray()
    Ainv_hat = _dense_Ahat_inv(S)
    Ahat = np.linalg.inv(Ainv_hat)
    n_p = B.shape[0]
    Sinv_hat = np.column_stack([S.Sinv(np.eye(n_p)[:, i]) for i in range(n_p)])
    Shat = np.linalg.inv(Sinv_hat)
    Khat = np.block([[Ahat, B.T], [B, B @ Ainv_hat @ B.T - Shat]])
    rng = np.random.default_rng(3)
    x = rng.standard_normal(K.shape[0])
    b = rng.standard_normal(K.shape[0])
    step = S.step(x, b)
    compact = x + np.linalg.solve(Khat, b - K @ x)
    assert np.allclose(step, compact, rtol=1e-10, atol=1e-10 * np.abs(compact).max())
    # the printed third update with the old pressure is not the compact form
    r_u = b[:nu] - A @ x[:nu] - B.T @ x[nu:]
    u_hat = x[:nu] + Ainv_hat @ r_u
    literal_u = x[:nu] + Ainv_hat @ (b[:nu] - A @ u_hat - B.T @ x[nu:])
    assert np.linalg.norm(literal_u - step[:nu]) > 1e-3 * np.linalg.norm(step[:nu])
    # spectral inequalities of the smoothing analysis: A_hat >= A, S_hat >= S~
    Ahs = 0.5 * (Ahat + Ahat.T)
    assert np.min(np.linalg.eigvalsh(Ahs - A)) > -1e-9 * np.abs(A).max()
    St = B @ Ainv_hat @ B.T
    Shs = 0.5 * (Shat + Shat.T)
    assert np.min(np.linalg.eigvalsh(Shs - St)) > -1e-9 * np.abs(St).max()
    # K_hat symmetric
    assert np.allclose(Khat, Khat.T, atol=1e-8 * np.abs(Khat).max())


def test_kA0_schur_diagonal_identity():
    mesh = BoxMesh(2, (4, 4), 2)
    asm = Assembled(mesh)
    S = LevelSmoother(asm, 0, 1, "d")
    n_p = asm.B.shape[0]
    diagS = np.array([S.S_tilde(np.eye(n_p)[:, i])[i] for i in range(n_p)])
    assert np.allclose(diagS, S.D_S / S.beta_A, rtol=1e-12)


def test_local_schur_diagonal_matches_hand_derivation():
    """D~_S_loc = sum_tau P_tau^T diag(B_tau diag(A_tau)^-1 B_tau^T) P_tau
    (Sec. 3.3.1) against exact rationals derived by hand from the 1D textbook
    element matrices (tests/golden/make_schur_loc_golden.py): non-square
    Cartesian cells, per-cell viscosity and a mass term, 2D and 3D.  Using
    the global diag(A), keeping the constrained velocity columns, or a
    transposed cell shape each moves entries by far more than the tolerance."""
    from fractions import Fraction
    g = _gold("schur_loc_golden.json")
    for cs in g["cases"]:
        d = len(cs["n"])
        hi = [float(Fraction(v)) for v in cs["box_hi"]]
        mu = np.array([float(Fraction(v)) for v in cs["mu_cell"]])
        mesh = BoxMesh(d, cs["n"], 2, lo=[0.0] * d, hi=hi, mu_cell=mu)
        asm = Assembled(mesh, gamma=float(Fraction(cs["gamma_rho"])), rho=1.0)
        ref = np.array([float(Fraction(v)) for v in cs["D_loc"]])
        D = schur_diagonal(asm, "loc")
        assert np.abs(D - ref).max() <= 1e-14 * np.abs(ref).max(), cs["name"]
        # the assembled-B choice is a different diagonal on the same mesh
        assert np.abs(schur_diagonal(asm, "d") - ref).max() > 0.1 * np.abs(ref).max()


def test_local_schur_diagonal_rotation_and_scaling_invariance():
    """D~_S_loc (Sec. 3.3.1) on cells given by their vertices: rotating and
    translating a mesh leaves every entry unchanged (sum_c (psi_i, d_c phi_j)^2
    and |grad phi_j|^2 are rotation invariant), and scaling it by s with no
    mass term multiplies every entry by s^d.  A Jacobian used untransposed
    or its determinant dropped breaks one of the two."""
    rng = np.random.default_rng(5)
    for d, n, ang in ((2, (3, 2), 0.7), (3, (2, 2, 1), 0.4)):
        if d == 2:
            R = np.array([[np.cos(ang), -np.sin(ang)], [np.sin(ang), np.cos(ang)]])
        else:
            ax = np.array([1.0, 2.0, 2.0]) / 3.0
            Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
            R = np.eye(3) + np.sin(ang) * Kx + (1 - np.cos(ang)) * Kx @ Kx
        mu = rng.uniform(0.5, 3.0, int(np.prod(n)))
        hi = [1.5, 1.0, 0.75][:d]
        base = BoxMesh(d, n, 2, lo=[0.0] * d, hi=hi, mu_cell=mu)
        ref = schur_diagonal(Assembled(base, gamma=2.0, rho=1.0), "loc")
        V = base.vertices @ R.T + 0.3
        rot = BoxMesh(d, n, 2, vertices=V, mu_cell=mu)
        D = schur_diagonal(Assembled(rot, gamma=2.0, rho=1.0), "loc")
        assert np.abs(D - ref).max() <= 1e-13 * np.abs(ref).max()
        s = 1.7
        ref0 = schur_diagonal(Assembled(base), "loc")
        big = BoxMesh(d, n, 2, vertices=s * V, mu_cell=mu)
        D0 = schur_diagonal(Assembled(big), "loc")
        assert np.abs(D0 - s ** d * ref0).max() <= 1e-13 * np.abs(s ** d * ref0).max()


def test_schur_diagonal_choices_are_spectrally_equivalent():
    # the three choices of Sec. 3.3.1 are all ~ diag(M_p) (their analysis)
    for n in (4, 8, 16):
        asm = Assembled(BoxMesh(2, (n, n), 2))
        Dp = schur_diagonal(asm, "p")
        for kind in ("d", "loc"):
            ratio = schur_diagonal(asm, kind) / Dp
            assert 0.05 < ratio.min() and ratio.max() < 20


# --------------------------------------------------------------------------
# transfers (Sec. 3.2)
# --------------------------------------------------------------------------
def test_q2_transfer_stencils_match_hand_values():
    g = _gold("transfer_stencils_q2.json")
    P = _field_prolongation([4], 2, 1).toarray()      # 1D, 4 coarse cells
    I = 4                                             # a coarse vertex node
    col = P[:, I]
    for off, w in zip(g["vertex_offsets"], g["vertex_weights_times_8"]):
        assert col[2 * I + off] == pytest.approx(w / 8, abs=1e-15)
    assert np.count_nonzero(np.abs(col) > 1e-15) == len(g["vertex_offsets"])
    I = 3                                             # a midpoint node
    col = P[:, I]
    for off, w in zip(g["mid_offsets"], g["mid_weights_times_4"]):
        assert col[2 * I + off] == pytest.approx(w / 4, abs=1e-15)
    Pq = _field_prolongation([4], 1, 1).toarray()
    col = Pq[:, 2]
    for off, w in zip(g["q1_offsets"], g["q1_weights_times_2"]):
        assert col[4 + off] == pytest.approx(w / 2, abs=1e-15)


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2)])
def test_prolongation_reproduces_coarse_polynomials(dim, k):
    mc, mf = make_hierarchy(dim, (2,) * dim, 2, k)
    P = prolongation(mc, mf)
    Xc, Xf = mc.velocity_node_coordinates(), mf.velocity_node_coordinates()
    # velocity: a polynomial of degree k per direction vanishing on the boundary
    g = lambda X: np.prod(X * (1 - X) * (0.3 + X) ** (k - 2), axis=1)
    u_c = np.concatenate([g(Xc)] * dim)
    # pressure: degree k-1 per direction, evaluated at pressure nodes (lattice of Q_{k-1})
    def pnodes(m):
        from oracle.fe import gll_points
        z = gll_points(k)
        idx = m._unflat(np.arange(m.n_pnode), m.p_dims)
        cell = np.minimum(idx // (k - 1), np.array(m.n) - 1)
        return (cell + z[idx - cell * (k - 1)]) / np.array(m.n)
    q = lambda X: np.prod(1.0 + X + 0.5 * X ** (k - 1), axis=1)
    x_c = np.concatenate([u_c, q(pnodes(mc))])
    x_f = np.concatenate([np.concatenate([g(Xf)] * dim), q(pnodes(mf))])
    assert np.allclose(P @ x_c, x_f, atol=1e-13)


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2)])
def test_galerkin_identity_on_nested_cartesian_meshes(dim, k):
    mc, mf = make_hierarchy(dim, (2,) * dim, 2, k)
    ac, af = Assembled(mc, gamma=3.0, c_p=0.5), Assembled(mf, gamma=3.0, c_p=0.5)
    P = prolongation(mc, mf)
    G = (P.T @ af.K @ P).toarray()
    Kc = ac.K.toarray()
    free = np.ones(Kc.shape[0], dtype=bool)
    free[ac.constrained] = False
    assert np.allclose(G[np.ix_(free, free)], Kc[np.ix_(free, free)], atol=1e-12 * np.abs(Kc).max())


# --------------------------------------------------------------------------
# coarse solve, outer solvers
# --------------------------------------------------------------------------
def test_bordered_coarse_solve():
    mg = Multigrid(make_hierarchy(2, (4, 4), 2, 2), gamma=1.0)
    a0 = mg.levels[0]
    rng = np.random.default_rng(1)
    b = rng.standard_normal(a0.K.shape[0])
    b[a0.constrained] = 0
    nu = a0.A.shape[0]
    b[nu:] -= b[nu:].mean()                        # consistent: 1^T b_p = 0
    x = mg.coarse_solve(b)
    assert np.linalg.norm(a0.K @ x - b) < 1e-12 * np.linalg.norm(b)
    assert abs((a0.Mp @ np.ones(a0.Mp.shape[0])) @ x[nu:]) < 1e-12 * np.linalg.norm(x)


def test_coarse_solve_with_pressure_mass_is_exact():
    """With C = c_p M_p (c_p > 0) constants leave the kernel of K_0: the coarse
    solve is the plain inverse, exact for any right-hand side, and the
    pressure mean is not forced to zero."""
    mg = Multigrid(make_hierarchy(2, (4, 4), 2, 2), gamma=1.0, c_p=0.3)
    a0 = mg.levels[0]
    rng = np.random.default_rng(3)
    b = rng.standard_normal(a0.K.shape[0])
    b[a0.constrained] = 0
    nu = a0.A.shape[0]
    x = mg.coarse_solve(b)
    assert np.linalg.norm(a0.K @ x - b) < 1e-12 * np.linalg.norm(b)
    # a pressure right-hand side with non-zero mean gives a pressure with non-zero mean
    assert abs((a0.Mp @ np.ones(a0.Mp.shape[0])) @ x[nu:]) > 1e-3 * np.linalg.norm(x[nu:])


def test_fgmres_matches_direct_solve_on_indefinite_system():
    rng = np.random.default_rng(2)
    n = 80
    M = rng.standard_normal((n, n)) + 4 * np.eye(n)
    M = M + M.T - 3 * np.diag(np.linspace(0, 8, n))    # symmetric indefinite
    b = rng.standard_normal(n)
    Ms = sp.csr_matrix(M)
    D = np.abs(np.diag(M)) + 1
    # full GMRES (restart >= n) is exact in at most n steps
    x, hist = fgmres(Ms, lambda v: v / D, b, rtol=1e-12, restart=n, maxit=n)
    assert np.allclose(x, np.linalg.solve(M, b), rtol=1e-9, atol=1e-9)
    assert hist[-1] <= 1e-12
    # restarted, on an SPD matrix with a varying (flexible) preconditioner
    Q = M @ M.T + n * np.eye(n)
    it = [0]

    def prec(v):
        it[0] += 1
        return v / (np.diag(Q) * (1.0 + 0.1 * (it[0] % 3)))
    x, hist = fgmres(sp.csr_matrix(Q), prec, b, rtol=1e-12, restart=10, maxit=2000)
    assert np.allclose(x, np.linalg.solve(Q, b), rtol=1e-9, atol=1e-10)


def test_rate_q_and_time_formula():
    hist = [1.0, 0.5, 0.1, 0.01, 0.001, 0.0001]
    assert rate_q(hist) == pytest.approx(0.1)
    assert time_to_reduce(2.0, 0.1) == pytest.approx(2.0)
    assert time_to_reduce(1.0, 0.01) == pytest.approx(0.5)


def test_sampled_rows_match_assembled_matrix():
    V = si.perturbed_box_vertices(4, dim=2, amplitude=0.2, seed=9)
    mesh = BoxMesh(2, (4, 4), 3, vertices=V, mu_cell=np.linspace(1, 3, 16))
    asm = Assembled(mesh, gamma=2.0, rho=0.5, c_p=0.3)
    x = si.uniform(mesh.n_total, 5)
    y = asm.K @ x
    dofs = np.arange(0, mesh.n_total, 7)
    ys = sample_Kx(mesh, x, dofs, gamma=2.0, rho=0.5, c_p=0.3)
    assert np.allclose(ys, y[dofs], rtol=1e-13, atol=1e-13)


def test_sampled_abs_rows_match_assembled_matrix():
    """(|K| |x|)_i of sampled rows, the scale of the componentwise parity
    measure, against the assembled matrix with its entries made absolute."""
    from oracle.rows import sample_abs_Kx
    V = si.perturbed_box_vertices(4, dim=2, amplitude=0.2, seed=9)
    mesh = BoxMesh(2, (4, 4), 3, vertices=V, mu_cell=np.linspace(1, 3, 16))
    asm = Assembled(mesh, gamma=2.0, rho=0.5, c_p=0.3)
    x = si.uniform(mesh.n_total, 5)
    dofs = np.arange(0, mesh.n_total, 3)
    ref = abs(asm.K) @ np.abs(x)
    assert np.allclose(sample_abs_Kx(mesh, x, dofs, gamma=2.0, rho=0.5, c_p=0.3), ref[dofs], rtol=1e-13, atol=0)


def test_sampled_diagonal_and_stencil_match_assembled_matrix():
    from oracle.rows import sample_diag_A, velocity_stencil
    V = si.perturbed_box_vertices(4, dim=2, amplitude=0.2, seed=9)
    mesh = BoxMesh(2, (4, 4), 2, vertices=V, mu_cell=np.linspace(1, 3, 16))
    asm = Assembled(mesh, gamma=2.0, rho=0.5)
    nu = asm.A.shape[0]
    dofs = np.arange(0, nu, 5)
    assert np.allclose(sample_diag_A(mesh, dofs, gamma=2.0, rho=0.5), asm.A.diagonal()[dofs], rtol=1e-14)
    # the stencil holds every column a free row of the constrained A reads
    Au = asm.A_unconstrained.tocsr()
    st = set(velocity_stencil(mesh, dofs).tolist())
    for g in dofs:
        assert set(Au.indices[Au.indptr[g]:Au.indptr[g + 1]].tolist()) <= st


# --------------------------------------------------------------------------
# the multigrid cycle as a linear iteration (Algorithm 1, Sec. 3.2)
# --------------------------------------------------------------------------
def _spectral_cheb_inverse(M, D, k, beta):
    """sigma Cheb(M, D, k) as a dense matrix from the eigen-decomposition of
    D^-1/2 M D^-1/2 and the closed-form residual polynomial s_k(t) = (1 -
    T_{k+1}(t)) / t of the Chebyshev iteration on [beta/2, beta] (Lemma 1)."""
    dh = 1.0 / np.sqrt(D)
    lam, Q = np.linalg.eigh(dh[:, None] * M * dh[None, :])
    alpha = beta / 2
    T = _cheb_T_closed(k + 1, (beta + alpha - 2 * lam) / (beta - alpha)) / \
        _cheb_T_closed(k + 1, np.array([(beta + alpha) / (beta - alpha)]))[0]
    return scaling_constant(k) * (dh[:, None] * (Q * ((1.0 - T) / lam)) @ Q.T * dh[None, :])


def _dense_smoother_inverse(asm, sm, kA, kS):
    """K_hat^-1 of the compact form of the smoother (Sec. 3.3.1):
    K_hat = [A_hat B^T; B B A_hat^-1 B^T - S_hat], A_hat, S_hat from the
    spectral form above with the smoother's own bounds beta_A, beta_S."""
    A, B, C = asm.A.toarray(), asm.B.toarray(), asm.C.toarray()
    Ai = _spectral_cheb_inverse(A, np.diag(A), kA, sm.beta_A)
    St = B @ Ai @ B.T + C
    Si = _spectral_cheb_inverse(0.5 * (St + St.T), sm.D_S, kS, sm.beta_S)
    Khat = np.block([[np.linalg.inv(Ai), B.T], [B, B @ Ai @ B.T - np.linalg.inv(Si)]])
    return np.linalg.inv(Khat)


def _coarse_pseudo_inverse(asm):
    """Level-0 solve as a matrix: the Moore-Penrose inverse of K_0, each
    column moved along the kernel vector (0, 1_p) to M_p-weighted pressure
    mean zero (the zero-mean reading of Q = L^2_0); K_0^-1 when C != 0."""
    K0 = asm.K.toarray()
    if asm.c_p != 0.0:
        return np.linalg.inv(K0)
    n, nu = K0.shape[0], asm.A.shape[0]
    X = np.linalg.pinv(K0, rcond=1e-13)
    kern = np.zeros(n)
    kern[nu:] = 1.0
    m = np.zeros(n)
    m[nu:] = asm.Mp @ np.ones(n - nu)
    return X - np.outer(kern, m @ X) / (m @ kern)


@pytest.mark.parametrize("levels,cycle,m,kA,kS,c_p", [(2, 1, 2, 1, 1, 0.0), (3, 1, 2, 1, 1, 0.0),
                                                     (3, 2, 1, 2, 1, 0.0), (2, 1, 1, 3, 2, 0.4)])
def test_cycle_is_the_multigrid_iteration(levels, cycle, m, kA, kS, c_p):
    """Algorithm 1 is the affine map x -> E_l x + N_l b with E_0 = 0, N_0 =
    K_0^+, and for l >= 1, with S = I - K_hat^-1 K_l (one smoothing step),
    S_m = S^m, N_m = sum_{i<m} S^i K_hat^-1, G = sum_{j<gamma_MG} E_{l-1}^j
    N_{l-1} (gamma_MG recursive calls from zero), CGC = I - P G P^T K_l
    (the coarse-grid correction of Sec. 3.2):
        E_l = S_m CGC S_m,   N_l = S_m (CGC N_m + P G P^T) + N_m.
    The oracle's cycle probed with unit vectors must equal these matrices: the
    error propagation everywhere, the right-hand-side map on consistent
    right-hand sides (b_p orthogonal to the constants).  Dropping either
    smoothing phase, the wrong number of recursive calls or a transposed
    transfer changes E by O(1)."""
    ms = make_hierarchy(2, (2, 2), levels, 2)
    mg = Multigrid(ms, gamma=3.0, c_p=c_p, k_A=kA, k_S=kS, smooth_steps=m, cycle_index=cycle)
    n = [mg.levels[l].K.shape[0] for l in range(levels)]
    E = [np.zeros((n[0], n[0]))]
    N = [_coarse_pseudo_inverse(mg.levels[0])]
    for l in range(1, levels):
        K = mg.levels[l].K.toarray()
        I = np.eye(n[l])
        Kh = _dense_smoother_inverse(mg.levels[l], mg.smoothers[l], kA, kS)
        S = I - Kh @ K
        Sm = np.linalg.matrix_power(S, m)
        Nm = sum(np.linalg.matrix_power(S, i) for i in range(m)) @ Kh
        P = mg.P[l].toarray()
        G = sum(np.linalg.matrix_power(E[l - 1], j) for j in range(cycle)) @ N[l - 1]
        CGC = I - P @ G @ P.T @ K
        E.append(Sm @ CGC @ Sm)
        N.append(Sm @ (CGC @ Nm + P @ G @ P.T) + Nm)
    L = levels - 1
    eye = np.eye(n[L])
    E_cyc = np.column_stack([mg.cycle(L, eye[:, j], np.zeros(n[L])) for j in range(n[L])])
    N_cyc = np.column_stack([mg.cycle(L, np.zeros(n[L]), eye[:, j]) for j in range(n[L])])
    assert np.abs(E_cyc - E[L]).max() <= 1e-12 * np.abs(E[L]).max()
    nu = mg.levels[L].A.shape[0]
    Pi = eye.copy()
    if c_p == 0.0:
        kern = np.zeros(n[L])
        kern[nu:] = 1.0
        Pi -= np.outer(kern, kern) / (kern @ kern)
    ref = N[L] @ Pi
    assert np.abs(N_cyc @ Pi - ref).max() <= 1e-12 * np.abs(ref).max()
    # the cycle without its post-smoothing is a different map
    assert np.abs(E_cyc - CGC @ Sm).max() > 1e-3 * np.abs(E[L]).max()


# --------------------------------------------------------------------------
# multigrid behaviour (Sec. 3.1, 4.3-4.6) -- qualitative
# --------------------------------------------------------------------------
def _mg_rate(n_levels, n_c=4, m=2, kA=1, kS=1, cycle=1, gamma=0.0, schur="d", dim=2):
    ms = make_hierarchy(dim, (n_c,) * dim, n_levels, 2)
    mg = Multigrid(ms, gamma=gamma, k_A=kA, k_S=kS, schur=schur, smooth_steps=m, cycle_index=cycle)
    asm = mg.levels[-1]
    f = si.nodal_random_f(dim, ms[-1].n_vnode, seed=2)
    b = asm.rhs_from_nodal_f(f)
    x, hist = stationary(asm.K, lambda x, b: mg.cycle(mg.L, x, b), b, rtol=1e-10, maxit=15)
    return rate_q(hist), hist


def test_mg_rate_is_level_independent():
    qs = [_mg_rate(L)[0] for L in (2, 3, 4)]
    assert max(qs) < 0.35, qs
    assert max(qs) < 2.0 * min(qs) + 0.02, qs


def test_mg_rate_improves_with_smoothing_steps_and_degree():
    q1 = _mg_rate(3, m=1)[0]
    q3 = _mg_rate(3, m=3)[0]
    assert q3 < q1
    q_low = _mg_rate(3, kA=0, kS=0, m=2)[0]
    q_high = _mg_rate(3, kA=3, kS=3, m=2)[0]
    assert q_high < q_low


def test_v_and_w_cycles_have_similar_rates_and_gamma_robustness():
    qv = _mg_rate(3, cycle=1)[0]
    qw = _mg_rate(3, cycle=2)[0]
    assert qw <= qv * 1.2 + 0.01 and qv <= 3 * qw + 0.05
    qg = _mg_rate(3, gamma=1e3)[0]
    assert qg < 2 * qv + 0.05


def test_mg_converges_with_every_schur_diagonal():
    for schur in ("d", "p", "loc", "exact"):
        q, hist = _mg_rate(2, n_c=2, schur=schur)
        assert q < 0.5 and hist[-1] < 1e-9 * hist[0], (schur, q)


def test_fgmres_with_mg_preconditioner_3d():
    ms = make_hierarchy(3, (2, 2, 2), 2, 2)
    mg = Multigrid(ms, k_A=1, k_S=1, smooth_steps=2)
    asm = mg.levels[-1]
    X = ms[-1].velocity_node_coordinates()
    b = asm.rhs_from_nodal_f(si.manufactured_f(X).T)
    x, hist = fgmres(asm.K, mg.precondition, b, rtol=1e-8)
    assert np.linalg.norm(b - asm.K @ x) <= 1e-8 * np.linalg.norm(b)
    assert len(hist) < 25


# --------------------------------------------------------------------------
# manufactured solutions: a-priori orders (Sec. 2)
# --------------------------------------------------------------------------
def _solve_direct(asm, b):
    n = asm.K.shape[0]
    nu = asm.A.shape[0]
    m = np.zeros(n)
    m[nu:] = asm.Mp @ np.ones(n - nu)
    Kb = sp.bmat([[asm.K, sp.csr_matrix(m[:, None])], [sp.csr_matrix(m[None, :]), None]]).tocsc()
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]


def _errors(mesh, x):
    d, k = mesh.dim, mesh.k
    cells = np.arange(mesh.ncell)
    cd = CellData(mesh, cells, nq_1d=k + 3)
    Nv = mesh.n_vnode
    vn = mesh.cell_velocity_nodes(cells)
    pn = mesh.cell_pressure_nodes(cells)
    u = x[:d * Nv].reshape(d, Nv)
    p = x[d * Nv:]
    Xq = cd.xq.reshape(-1, d)
    ue = si.manufactured_u(Xq).reshape(len(cells), -1, d)
    ge = si.manufactured_grad_u(Xq).reshape(len(cells), -1, d, d)
    pe = si.manufactured_p(Xq).reshape(len(cells), -1)
    uh = np.einsum("iq,cai->cqa", cd.phi, u[:, vn].transpose(1, 0, 2))
    gh = np.einsum("ciqb,cai->cqab", cd.grad, u[:, vn].transpose(1, 0, 2))
    ph = np.einsum("iq,ci->cq", cd.psi, p[pn])
    vol = cd.JxW.sum()
    ph = ph - (ph * cd.JxW).sum() / vol
    pe = pe - (pe * cd.JxW).sum() / vol
    eu = np.sqrt(np.sum(((uh - ue) ** 2).sum(-1) * cd.JxW))
    eg = np.sqrt(np.sum(((gh - ge) ** 2).sum((-1, -2)) * cd.JxW))
    ep = np.sqrt(np.sum((ph - pe) ** 2 * cd.JxW))
    return eu, eg, ep


@pytest.mark.parametrize("dim,k,ns", [(2, 2, (4, 8, 16, 32)), (2, 3, (4, 8, 16)), (3, 2, (2, 4, 8))])
def test_manufactured_convergence_orders(dim, k, ns):
    errs = []
    for n in ns:
        mesh = BoxMesh(dim, (n,) * dim, k)
        asm = Assembled(mesh, keep_local=False)
        b = rhs_closed_form(mesh, lambda X: si.manufactured_f(X))
        x = _solve_direct(asm, b)
        errs.append(_errors(mesh, x))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])[-1]
    # velocity L2 ~ k+1, velocity H1 ~ k, pressure L2 ~ k
    assert rates[0] > k + 1 - 0.3, (errs, rates)
    assert rates[1] > k - 0.3, (errs, rates)
    assert rates[2] > k - 0.3, (errs, rates)
