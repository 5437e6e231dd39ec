"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no finite-element or solver arithmetic: only random numbers
(NumPy PCG64 streams), closed-form analytic fields, and mesh-vertex
perturbations on the box lattice.  Discretisation-dependent quantities (node
coordinates, DoF counts) are passed in by the caller, each side computing
its own.

Workloads (unit box, homogeneous Dirichlet velocity):
  * 2D Q2-Q1 16^2, 3 levels, mu = 1, gamma = 0, manufactured solution;
  * 2D Q2-Q1 512^2, 7 levels, mu = rho = 1, gamma = 1e3, nodal f ~ U[-1,1] (seed 2);
  * 3D Q2-Q1 64^3, 6 levels, mu = 1, gamma = 0, manufactured solution;
  * 3D Q3-Q2 32^3, 5 levels, perturbed interior vertices (seed 4), per-cell
    mu = exp(sum of 8 Fourier modes) scaled to [1, 100] (seed 5).
The paper's benchmark problems (driven cavity, flow around a cylinder) need
non-homogeneous boundary data or curved geometry; these box problems with the
same element pair, comparable DoF counts and the same (mu, gamma) regime
stand in for them.
"""
import numpy as np


def uniform(n, seed, lo=-1.0, hi=1.0):
    """n values U[lo, hi) from PCG64(seed)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=int(n))


def nodal_random_f(dim, n_vnode, seed=2):
    """Random nodal body force, one value per velocity node and component,
    U[-1, 1], shape (dim, n_vnode)."""
    return uniform(dim * n_vnode, seed).reshape(dim, n_vnode)


# ---------------------------------------------------------------------------
# closed-form manufactured solution: u = curl psi (div-free, u = grad u = 0 on
# the boundary of the unit box), p = prod cos(pi x_a) (zero mean)
# ---------------------------------------------------------------------------
def _S(t, order):
    """Derivatives of S(t) = sin^2(pi t)."""
    pi = np.pi
    if order == 0:
        return np.sin(pi * t) ** 2
    if order == 1:
        return pi * np.sin(2 * pi * t)
    if order == 2:
        return 2 * pi ** 2 * np.cos(2 * pi * t)
    if order == 3:
        return -4 * pi ** 3 * np.sin(2 * pi * t)
    raise ValueError(order)


def _dpsi(X, orders):
    out = np.ones(X.shape[0])
    for a, o in enumerate(orders):
        out = out * _S(X[:, a], o)
    return out


def _curl_terms(dim):
    """u_c = sum_(sign, a) sign * d_a psi  (2D: psi scalar, 3D: Psi = (psi, psi, psi))."""
    if dim == 2:
        return [[(+1, 1)], [(-1, 0)]]
    return [[(+1, 1), (-1, 2)], [(+1, 2), (-1, 0)], [(+1, 0), (-1, 1)]]


def manufactured_u(X):
    X = np.atleast_2d(X)
    dim = X.shape[1]
    out = np.zeros((X.shape[0], dim))
    for c, terms in enumerate(_curl_terms(dim)):
        for sgn, a in terms:
            o = [0] * dim
            o[a] = 1
            out[:, c] += sgn * _dpsi(X, o)
    return out


def manufactured_grad_u(X):
    """G[n, c, b] = d u_c / d x_b."""
    X = np.atleast_2d(X)
    dim = X.shape[1]
    out = np.zeros((X.shape[0], dim, dim))
    for c, terms in enumerate(_curl_terms(dim)):
        for sgn, a in terms:
            for b in range(dim):
                o = [0] * dim
                o[a] += 1
                o[b] += 1
                out[:, c, b] += sgn * _dpsi(X, o)
    return out


def manufactured_laplace_u(X):
    X = np.atleast_2d(X)
    dim = X.shape[1]
    out = np.zeros((X.shape[0], dim))
    for c, terms in enumerate(_curl_terms(dim)):
        for sgn, a in terms:
            for b in range(dim):
                o = [0] * dim
                o[a] += 1
                o[b] += 2
                out[:, c] += sgn * _dpsi(X, o)
    return out


def manufactured_p(X):
    X = np.atleast_2d(X)
    return np.prod(np.cos(np.pi * X), axis=1)


def manufactured_grad_p(X):
    X = np.atleast_2d(X)
    dim = X.shape[1]
    out = np.zeros((X.shape[0], dim))
    for b in range(dim):
        term = -np.pi * np.sin(np.pi * X[:, b])
        for a in range(dim):
            if a != b:
                term = term * np.cos(np.pi * X[:, a])
        out[:, b] = term
    return out


def manufactured_f(X, mu=1.0, gamma=0.0, rho=1.0):
    """f = -mu Laplace u + gamma rho u + grad p, shape (n, dim)."""
    return (-mu * manufactured_laplace_u(X) + gamma * rho * manufactured_u(X)
            + manufactured_grad_p(X))


# ---------------------------------------------------------------------------
# perturbed vertices and per-cell viscosity (3D Q3-Q2 workload)
# ---------------------------------------------------------------------------
def perturbed_box_vertices(n, dim=3, amplitude=0.2, seed=4):
    """Vertices of the unit-box lattice with n cells per direction (an int, or
    one count per direction), interior vertices moved by U[-amplitude h_a,
    amplitude h_a] in coordinate a; x fastest."""
    ns = [int(n)] * dim if np.isscalar(n) else [int(v) for v in n][:dim]
    axes = [np.linspace(0.0, 1.0, v + 1) for v in ns]
    grids = np.meshgrid(*axes, indexing="ij")
    V = np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids], axis=1)
    idx = np.indices(tuple(v + 1 for v in ns)).reshape(dim, -1)[::-1].T
    interior = np.all((idx > 0) & (idx < np.array(ns)), axis=1)
    rng = np.random.default_rng(seed)
    h = 1.0 / np.array(ns, dtype=np.float64)
    shift = rng.uniform(-amplitude * h, amplitude * h, size=V.shape)
    V[interior] += shift[interior]
    return V


def fourier_log_viscosity(n, dim=3, modes=8, mu_min=1.0, mu_max=100.0, seed=5):
    """Per-cell viscosity mu = exp(g(x_tau)), g a sum of `modes` random Fourier
    modes at the cell centres of the n^dim lattice, affinely rescaled so that
    log mu spans [log mu_min, log mu_max]; cells x fastest."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(modes)
    kv = []
    while len(kv) < modes:
        cand = rng.integers(0, 4, size=dim)
        if np.any(cand != 0):
            kv.append(cand)
    kv = np.array(kv)
    phase = rng.uniform(0.0, 2 * np.pi, size=modes)
    idx = np.indices((n,) * dim).reshape(dim, -1)[::-1].T
    xc = (idx + 0.5) / n
    g = np.zeros(xc.shape[0])
    for m in range(modes):
        g += a[m] * np.cos(2 * np.pi * xc @ kv[m] + phase[m])
    g = (g - g.min()) / (g.max() - g.min())
    return np.exp(np.log(mu_min) + g * (np.log(mu_max) - np.log(mu_min)))


def smooth_random_field(X, seed=6, modes=6):
    """A seeded smooth vector field on the unit box vanishing on its boundary
    (product of sines times random low-frequency modes), shape (n, dim)."""
    X = np.atleast_2d(X)
    dim = X.shape[1]
    rng = np.random.default_rng(seed)
    bubble = np.prod(np.sin(np.pi * X), axis=1)
    out = np.zeros((X.shape[0], dim))
    for c in range(dim):
        for _ in range(modes):
            kv = rng.integers(0, 3, size=dim)
            ph = rng.uniform(0, 2 * np.pi)
            out[:, c] += rng.standard_normal() * np.cos(2 * np.pi * X @ kv + ph)
        out[:, c] *= bubble
    return out


# ---------------------------------------------------------------------------
# batches of independent instances (2D generalized Stokes)
# ---------------------------------------------------------------------------
def batch_instances(count=64, n_min=32, n_max=512, gamma_max=1e4, seed=7):
    """Side counts drawn log-uniformly in [n_min, n_max] and snapped to the
    nearest c 2^j with c in {4, 5, 6, 7} (coarsest mesh c x c, j + 1 levels),
    gamma ~ U[0, gamma_max]; returns a list of dicts (n, c, levels, gamma)."""
    rng = np.random.default_rng(seed)
    draws = np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=count))
    gammas = rng.uniform(0.0, gamma_max, size=count)
    cands = sorted({(c * 2 ** j, c, j) for c in (4, 5, 6, 7) for j in range(0, 12)})
    out = []
    for v, g in zip(draws, gammas):
        n, c, j = min(cands, key=lambda t: (abs(t[0] - v), t[0]))
        out.append(dict(n=n, c=c, levels=j + 1, gamma=float(g)))
    return out
