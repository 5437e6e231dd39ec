"""Outer iterations (oracle; test infrastructure only).

Section 4.1 protocol: stationary multigrid iterations x^{j+1} = MG(x^j, b) from
x^0 = 0 until the Euclidean residual r^j = ||b - K x^j|| has dropped by the
requested factor (at most 15 iterations in the paper), with the rate
q = (r^j / r^{j-3})^{1/3} over the last three steps and the time-to-reduction
T(eps) = T_iter log(eps) / log(q).

FGMRES: the paper has no Krylov outer loop; the right-preconditioned flexible
GMRES(m) with classical Gram-Schmidt applied twice is the outer solver in
which an FP64 or FP32 multigrid cycle serves as the (possibly inexact)
preconditioner.  Textbook algorithm (Saad, flexible GMRES), FP64 throughout.
"""
import math
import numpy as np


def rate_q(history):
    """Average reduction of the last three steps (fewer when fewer exist)."""
    j = len(history) - 1
    if j <= 0:
        return float("nan")
    s = min(3, j)
    if history[j - s] == 0.0:
        return 0.0
    return (history[j] / history[j - s]) ** (1.0 / s)


def time_to_reduce(t_iter, q, eps=0.1):
    return t_iter * math.log(eps) / math.log(q)


def stationary(K, cycle, b, rtol=1e-10, maxit=15, x0=None):
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r0 = np.linalg.norm(b - K @ x)
    hist = [r0]
    for _ in range(maxit):
        x = cycle(x, b)
        hist.append(np.linalg.norm(b - K @ x))
        if hist[-1] <= rtol * r0:
            break
    return x, hist


def fgmres(K, precond, b, x0=None, rtol=1e-8, restart=30, maxit=300):
    """Right-preconditioned flexible GMRES(restart); returns x, residual history
    (relative to ||b||, one entry per iteration plus the initial one)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, [0.0]
    r = b - K @ x
    beta = np.linalg.norm(r)
    hist = [beta / bnorm]
    it = 0
    while it < maxit and beta / bnorm > rtol:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = K @ Z[j]
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            H[:j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= rtol or it >= maxit:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:]) / H[i, i]
        x = x + Z[:j_done].T @ y
        r = b - K @ x
        beta = np.linalg.norm(r)
        hist[-1] = beta / bnorm
    return x, hist
