"""One-dimensional finite-element ingredients (oracle; test infrastructure only).

Section 2 builds the Taylor-Hood spaces from tensor-product nodal bases on the
reference cell (0,1)^d: velocity Q_k, pressure Q_{k-1}, k >= 2.  The paper
does not fix the node positions for k >= 3 nor the quadrature rule; the
readings used here are
  * nodes: Gauss-Lobatto-Legendre points on [0,1] (k+1 for velocity, k for
    pressure); for k = 2 these are the equidistant points {0, 1/2, 1};
  * quadrature: Gauss-Legendre with k+1 points per direction, which integrates
    every term of a, b and the mass matrices exactly on affine cells.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(npts):
    """Gauss-Lobatto-Legendre points on [0,1]: the end points and the roots of
    P'_{npts-1} (Legendre polynomial derivative), mapped from [-1,1]."""
    if npts < 2:
        raise ValueError("need at least two GLL points")
    n = npts - 1
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    interior = np.sort(npleg.legroots(npleg.legder(coef))) if n >= 2 else np.zeros(0)
    x = np.concatenate(([-1.0], interior, [1.0]))
    return 0.5 * (x + 1.0)


def gauss_rule(nq):
    """Gauss-Legendre rule with nq points on [0,1] (points, weights)."""
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """Matrix V[i, q] = l_i(x_q) of the Lagrange polynomials through `nodes`."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((n, len(x)))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """Matrix G[i, q] = l_i'(x_q), by the product rule on the same products."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    G = np.zeros((n, len(x)))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term = term * (x - nodes[j]) / (nodes[i] - nodes[j])
            G[i] += term
    return G


def tensor_multi_indices(npts, dim):
    """Local node multi-indices of a tensor-product cell, x fastest:
    row r = (a_x, a_y[, a_z]) with r = a_x + npts*(a_y + npts*a_z)."""
    idx = np.indices((npts,) * dim).reshape(dim, -1)[::-1].T
    return idx.copy()


def reference_basis(nodes_1d, dim, qpts_1d):
    """Values and reference gradients of the tensor-product Lagrange basis at
    the tensor-product quadrature points.

    Returns (phi[nloc, nq], dphi[nloc, nq, dim]) with both local nodes and
    quadrature points ordered x fastest."""
    V = lagrange_values(nodes_1d, qpts_1d)
    G = lagrange_derivatives(nodes_1d, qpts_1d)
    loc = tensor_multi_indices(len(nodes_1d), dim)
    qid = tensor_multi_indices(len(qpts_1d), dim)
    nloc, nq = len(loc), len(qid)
    phi = np.ones((nloc, nq))
    dphi = np.ones((nloc, nq, dim))
    for a in range(dim):
        va = V[loc[:, a]][:, qid[:, a]]
        ga = G[loc[:, a]][:, qid[:, a]]
        phi *= va
        for b in range(dim):
            dphi[:, :, b] *= ga if a == b else va
    return phi, dphi


def quadrature_weights(wq_1d, dim):
    qid = tensor_multi_indices(len(wq_1d), dim)
    w = np.ones(len(qid))
    for a in range(dim):
        w *= np.asarray(wq_1d)[qid[:, a]]
    return w
