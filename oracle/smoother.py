"""Scaled Chebyshev-Jacobi inexact symmetric Uzawa smoother (oracle; test
infrastructure only).

Section 3.3.1 and Algorithm 2 (smoother setup):
  A^-1_hat = sigma * Cheb(A, D_A, k_A),  D_A = diag(A),
  S^-1_hat = tau * Cheb(S~, D~_S, k_S),  S~ = B A^-1_hat B^T + C,
  [alpha, beta] = [beta/2, beta], beta ~ lambda_max(D^-1 M),
  sigma, tau = C_{k+1}(s) / (1 + C_{k+1}(s)),  s = (beta+alpha)/(beta-alpha) = 3,
with Cheb(M, D, k) = s_k(D^-1 M) D^-1, s_k(t) = (1 - T_{k+1}(t)) / t, evaluated by
the three-term Chebyshev-acceleration recurrence the paper cites (Saad).

The Schur diagonals are the three choices of Section 3.3.1: D~_{S_d} =
diag(B diag(A)^-1 B^T), D~_{S_p} = diag(M_p), D~_{S_loc} = sum over cells of
diag(B_tau diag(A_tau)^-1 B_tau^T); plus the exact diag(S~) by probing (tiny
meshes).  Readings: constrained velocity columns are excluded everywhere
(they are zero columns of the constrained B); with C != 0, diag(C) is added.

The smoother step (Section 1, the three inexact symmetric Uzawa updates) is
taken in the form that matches the compact form x <- x + K_hat^-1 (b - K x)
with K_hat = [A_hat B^T; B B A_hat^-1 B^T - S_hat] of Section 3.3.1.  The
third update as printed (with the old pressure) contradicts that compact form;
the reading used is u^{j+1} = u_hat - A_hat^-1 B^T (p^{j+1} - p^j).

Eigenvalue estimate (the paper only says a close approximation of lambda_max
is used): Lanczos in the D inner product without reorthogonalisation, from a
SplitMix64 start vector, beta = safety * theta_max.
"""
import numpy as np
from numpy.polynomial import chebyshev as npcheb
import scipy.sparse as sp

LANCZOS_STEPS = 30
LANCZOS_SAFETY = 1.02
LANCZOS_SEED_A = 1234
LANCZOS_SEED_S = 4321


def chebyshev_first_kind(n, x):
    """C_n(x), the Chebyshev polynomial of the first kind."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npcheb.chebval(x, c)


def scaling_constant(k, sbar=3.0):
    """c_1 of Lemma 1 = C_{k+1}(s) / (1 + C_{k+1}(s)); sigma and tau of Algorithm 2."""
    C = chebyshev_first_kind(k + 1, sbar)
    return C / (1.0 + C)


def chebyshev_apply(matvec, dinv, r, k, beta, alpha=None):
    """Cheb(M, D, k) r: k applications of M, result s_k(D^-1 M) D^-1 r."""
    alpha = 0.5 * beta if alpha is None else alpha
    theta = 0.5 * (beta + alpha)
    delta = 0.5 * (beta - alpha)
    s1 = theta / delta
    rho = 1.0 / s1
    x = np.zeros_like(r)
    res = r.copy()
    d = dinv * res / theta
    for _ in range(k):
        x = x + d
        res = res - matvec(d)
        rho_new = 1.0 / (2.0 * s1 - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * res)
        rho = rho_new
    return x + d


def splitmix64_u64(seed, n):
    """The first n outputs of SplitMix64 (Steele, Lea, Flood 2014) for a
    given seed, as a counter-based generator: output i (i = 1..n) mixes
    z = seed + i * 0x9E3779B97F4A7C15 by two xor-shift-multiply rounds."""
    mask = (1 << 64) - 1
    out = []
    for i in range(1, n + 1):
        z = (seed + i * 0x9E3779B97F4A7C15) & mask
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


def splitmix64_uniform(seed, n):
    """n numbers in [-1, 1): top 53 bits of each SplitMix64 output / 2^53,
    mapped affinely."""
    return np.array([2.0 * ((z >> 11) / float(1 << 53)) - 1.0 for z in splitmix64_u64(seed, n)])


def lanczos_max(matvec, dvec, v0, steps=LANCZOS_STEPS):
    """Largest Ritz value of D^-1 M after `steps` Lanczos steps in the D inner
    product <x, y>_D = x^T D y (D diagonal, given as a vector)."""
    q = v0 / np.sqrt(np.dot(v0, dvec * v0))
    q_prev = np.zeros_like(q)
    alphas, betas = [], []
    b_prev = 0.0
    for j in range(min(steps, len(v0))):
        w = matvec(q) / dvec
        a = np.dot(w, dvec * q)
        w = w - a * q - b_prev * q_prev
        alphas.append(a)
        b = np.sqrt(max(np.dot(w, dvec * w), 0.0))
        if b <= 1e-14 * abs(a):
            break
        betas.append(b)
        q_prev, q = q, w / b
        b_prev = b
    m = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:m - 1], 1) + np.diag(betas[:m - 1], -1)
    return float(np.max(np.linalg.eigvalsh(T)))


class LevelSmoother:
    """Smoother ingredients of one level (Algorithm 2) on assembled matrices."""

    def __init__(self, asm, k_A=1, k_S=1, schur="d", beta_A=None, beta_S=None):
        self.asm = asm
        self.A, self.B, self.C = asm.A, asm.B, asm.C
        self.nu = self.A.shape[0]
        self.k_A, self.k_S = k_A, k_S
        self.sigma = scaling_constant(k_A)
        self.tau = scaling_constant(k_S)
        self.D_A = self.A.diagonal().copy()
        self.dinv_A = 1.0 / self.D_A
        if beta_A is None:
            v0 = splitmix64_uniform(LANCZOS_SEED_A, self.nu) * asm.free_u
            beta_A = LANCZOS_SAFETY * lanczos_max(lambda v: self.A @ v, self.D_A, v0)
        self.beta_A = beta_A
        self.D_S = schur_diagonal(asm, schur, self if schur == "exact" else None)
        self.dinv_S = 1.0 / self.D_S
        if beta_S is None:
            v0 = splitmix64_uniform(LANCZOS_SEED_S, self.B.shape[0])
            beta_S = LANCZOS_SAFETY * lanczos_max(self.S_tilde, self.D_S, v0)
        self.beta_S = beta_S

    # A_hat^-1 and S_hat^-1 -------------------------------------------------
    def Ainv(self, r):
        return self.sigma * chebyshev_apply(lambda v: self.A @ v, self.dinv_A, r, self.k_A, self.beta_A)

    def S_tilde(self, q):
        return self.B @ self.Ainv(self.B.T @ q) + self.C @ q

    def Sinv(self, r):
        return self.tau * chebyshev_apply(self.S_tilde, self.dinv_S, r, self.k_S, self.beta_S)

    # one inexact symmetric Uzawa step -------------------------------------
    def step(self, x, b):
        nu = self.nu
        u, p = x[:nu], x[nu:]
        f, g = b[:nu], b[nu:]
        r_u = f - self.A @ u - self.B.T @ p
        u_hat = u + self.Ainv(r_u)
        r_p = self.B @ u_hat - self.C @ p - g
        dp = self.Sinv(r_p)
        u_new = u_hat - self.Ainv(self.B.T @ dp)
        return np.concatenate([u_new, p + dp])

    def smooth(self, x, b, steps):
        for _ in range(steps):
            x = self.step(x, b)
        return x


def schur_diagonal(asm, kind, smoother=None):
    """D~_S for the choices of Section 3.3.1 (plus diag(C))."""
    B = asm.B
    if kind == "d":
        D_A = asm.A.diagonal()
        D = np.asarray(B.multiply(B) @ (1.0 / D_A)).ravel()
    elif kind == "p":
        D = asm.Mp.diagonal().copy()
    elif kind == "loc":
        if asm.form != "grad":
            raise ValueError("the local Schur diagonal is defined here for the gradient form only")
        mesh = asm.mesh
        cells = np.arange(mesh.ncell)
        vn = mesh.cell_velocity_nodes(cells)
        pn = mesh.cell_pressure_nodes(cells)
        free_node = (~mesh.velocity_boundary_nodes()).astype(np.float64)
        fr = free_node[vn]                                            # (nc, nv)
        Bt = asm.local_B                                              # (nc, np, d, nv)
        loc = np.einsum("cpaj,cj->cp", Bt ** 2, fr / asm.local_Adiag)
        D = np.zeros(mesh.n_pnode)
        np.add.at(D, pn.ravel(), loc.ravel())
    elif kind == "exact":
        n = B.shape[0]
        D = np.zeros(n)
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            D[i] = (B @ smoother.Ainv(B.T @ e))[i]
        return D + asm.C.diagonal()
    else:
        raise ValueError(kind)
    return D + asm.C.diagonal()
