"""Monolithic geometric multigrid (oracle; test infrastructure only).

Algorithm 1 with cycle index gamma_MG (1: V-cycle, 2: W-cycle; the paper
mostly uses W and recommends V in practice, Section 4.3), m pre- and m
post-smoothing steps of the Uzawa smoother, transfers of Section 3.2, and a
direct solve on level 0 (Section 4.1: assembled coarse matrix, direct method).
Reading of Algorithm 1: on level 0 the exact solve is the whole cycle (it
returns without smoothing).

Coarse solve reading: for C = 0 the pressure is only fixed up to a constant
(Q = L^2_0 in Section 2), so level 0 solves the bordered system
[K_0 m; m^T 0] with m = (0, M_p 1), i.e. the discrete zero-mean condition on
p.  With C = c_p M_p, c_p > 0, constants are no longer in the kernel of K_0,
which is regular and solved as it is.
"""
import numpy as np

from .assemble import Assembled
from .smoother import LevelSmoother
from .transfer import prolongation


class Multigrid:
    def __init__(self, meshes, mu=1.0, gamma=0.0, rho=1.0, c_p=0.0,
                 k_A=1, k_S=1, schur="d", smooth_steps=2, cycle_index=1, betas=None, form="grad"):
        self.meshes = meshes
        self.L = len(meshes) - 1
        self.m = smooth_steps
        self.cycle_index = cycle_index
        self.levels = [Assembled(me, mu, gamma, rho, c_p, form=form) for me in meshes]
        self.P = [None] + [prolongation(meshes[l - 1], meshes[l]) for l in range(1, self.L + 1)]
        self.smoothers = [None]
        for l in range(1, self.L + 1):
            bA, bS = (None, None) if betas is None else betas[l]
            self.smoothers.append(LevelSmoother(self.levels[l], k_A, k_S, schur, bA, bS))
        K0 = self.levels[0].K.toarray()
        n0 = K0.shape[0]
        nu0 = self.levels[0].A.shape[0]
        self.bordered = c_p == 0.0
        if self.bordered:
            mvec = np.zeros(n0)
            mvec[nu0:] = self.levels[0].Mp @ np.ones(n0 - nu0)
            Kb = np.zeros((n0 + 1, n0 + 1))
            Kb[:n0, :n0] = K0
            Kb[:n0, n0] = mvec
            Kb[n0, :n0] = mvec
            self.K0_bordered = Kb
        else:
            self.K0_bordered = K0

    def K(self, l):
        return self.levels[l].K

    def coarse_solve(self, b0):
        if not self.bordered:
            return np.linalg.solve(self.K0_bordered, b0)
        rhs = np.concatenate([b0, [0.0]])
        return np.linalg.solve(self.K0_bordered, rhs)[:-1]

    def cycle(self, l, x, b):
        if l == 0:
            return self.coarse_solve(b)
        S = self.smoothers[l]
        x = S.smooth(x, b, self.m)
        r = b - self.levels[l].K @ x
        rc = self.P[l].T @ r
        w = np.zeros_like(rc)
        for _ in range(self.cycle_index):
            w = self.cycle(l - 1, w, rc)
        x = x + self.P[l] @ w
        x = S.smooth(x, b, self.m)
        return x

    def precondition(self, v):
        """One cycle on the finest level with zero initial guess."""
        return self.cycle(self.L, np.zeros_like(v), v)

    def betas(self):
        return [None] + [(s.beta_A, s.beta_S) for s in self.smoothers[1:]]


def pressure_mean_free(asm, x):
    """Remove the M_p-weighted mean of the pressure part of x."""
    nu = asm.A.shape[0]
    p = x[nu:]
    one = np.ones_like(p)
    w = asm.Mp @ one
    out = x.copy()
    out[nu:] = p - np.dot(w, p) / np.dot(w, one)
    return out
