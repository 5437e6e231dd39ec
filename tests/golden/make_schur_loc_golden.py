"""Writes schur_loc_golden.json: the local Schur-complement diagonal of
Sec. 3.3.1,

    D~_S_loc = sum_tau P_tau^T diag(B_tau diag(A_tau)^-1 B_tau^T) P_tau,

on small Cartesian Q2-Q1 meshes, in exact rational arithmetic, derived by
hand from the closed-form 1D element matrices of element_matrices_1d.json.
It imports nothing from the oracle or the library: the cell matrices are the
tensor-product forms of a Cartesian cell [0,h_x] x [0,h_y] (x [0,h_z]):

  velocity node (i_x, i_y[, i_z]) in {0,1,2}^d, pressure node (q_x, q_y[, q_z])
  in {0,1}^d (x fastest),

  (A_tau)_{ii} = mu_tau * sum_a K1(h_a)[i_a,i_a] prod_{b != a} M1(h_b)[i_b,i_b]
                 + gamma rho prod_a M1(h_a)[i_a,i_a]          (form a, Sec. 2)
  (B_tau)_{q,(c,i)} = - G12[q_c,i_c] prod_{b != c} N12(h_b)[q_b,i_b]
                                                            (form b, B = -div)

with K1(h) = S/(3h), M1(h) = M h/30 (Q2), G12 = D/6 (Q1 value x Q2
derivative, h-free), N12(h) = N h/6 (Q1 x Q2 mass).  Velocity columns of
boundary nodes are left out (they are zero columns of the constrained B).

Run from the repository root:  python tests/golden/make_schur_loc_golden.py
"""
import itertools
import json
import os
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))


def one_d():
    with open(os.path.join(HERE, "element_matrices_1d.json")) as fh:
        g = json.load(fh)
    S = [[F(v) for v in r] for r in g["q2_stiffness_times_3h"]]
    M = [[F(v) for v in r] for r in g["q2_mass_times_30_over_h"]]
    D = [[F(v) for v in r] for r in g["q1_q2_derivative_times_6"]]
    N = [[F(v) for v in r] for r in g["q1_q2_mass_times_6_over_h"]]
    K1 = lambda h: [[s / (3 * h) for s in r] for r in S]
    M1 = lambda h: [[m * h / 30 for m in r] for r in M]
    G12 = [[v / 6 for v in r] for r in D]
    N12 = lambda h: [[v * h / 6 for v in r] for r in N]
    return K1, M1, G12, N12


def schur_loc(n, box_hi, mu_cell, gamma_rho):
    """D~_S_loc as a list of Fractions over the pressure lattice (x fastest)."""
    K1, M1, G12, N12 = one_d()
    d = len(n)
    h = [F(box_hi[a]) / n[a] for a in range(d)]
    vdims = [2 * n[a] + 1 for a in range(d)]
    pdims = [n[a] + 1 for a in range(d)]

    def flat(idx, dims):
        out, stride = 0, 1
        for a in range(d):
            out += idx[a] * stride
            stride *= dims[a]
        return out

    n_p = 1
    for a in range(d):
        n_p *= pdims[a]
    D = [F(0)] * n_p
    cells = list(itertools.product(*[range(n[a]) for a in range(d)][::-1]))   # slowest axis first
    for ci, cidx_rev in enumerate(cells):
        c = list(cidx_rev[::-1])                                 # (c_x, c_y[, c_z])
        mu = F(mu_cell[ci])
        loc_v = list(itertools.product(*[range(3)] * d))         # reversed order tuples
        loc_p = list(itertools.product(*[range(2)] * d))
        for qrev in loc_p:
            q = list(qrev[::-1])
            s = F(0)
            for irev in loc_v:
                i = list(irev[::-1])
                glob = [2 * c[a] + i[a] for a in range(d)]
                if any(glob[a] == 0 or glob[a] == vdims[a] - 1 for a in range(d)):
                    continue                                      # constrained column
                a_ii = F(0)
                for a in range(d):
                    t = K1(h[a])[i[a]][i[a]]
                    for b in range(d):
                        if b != a:
                            t *= M1(h[b])[i[b]][i[b]]
                    a_ii += mu * t
                m = F(gamma_rho)
                for a in range(d):
                    m *= M1(h[a])[i[a]][i[a]]
                a_ii += m
                for comp in range(d):
                    bq = -G12[q[comp]][i[comp]]
                    for b in range(d):
                        if b != comp:
                            bq *= N12(h[b])[q[b]][i[b]]
                    s += bq * bq / a_ii
            gp = [c[a] + q[a] for a in range(d)]
            D[flat(gp, pdims)] += s
    return D


CASES = [
    dict(name="2d_3x3", n=[3, 3], box_hi=["9/10", "3/5"], gamma_rho="1",
         mu_cell=[str(F(4 + c, 4)) for c in range(9)]),
    dict(name="3d_2x2x2", n=[2, 2, 2], box_hi=["1", "3/4", "1/2"], gamma_rho="3",
         mu_cell=[str(F(2 + c, 2)) for c in range(8)]),
]


def main():
    out = {"_source": ("Local Schur diagonal of Sec. 3.3.1 on Cartesian Q2-Q1 meshes, exact rationals, "
                       "hand-derived from element_matrices_1d.json by tests/golden/make_schur_loc_golden.py "
                       "(tensor-product cell matrices; constrained velocity columns left out). "
                       "Box [0, box_hi], per-cell mu (x fastest), gamma*rho as given."),
           "cases": []}
    for cs in CASES:
        D = schur_loc(cs["n"], [F(v) for v in cs["box_hi"]], [F(v) for v in cs["mu_cell"]], F(cs["gamma_rho"]))
        rec = dict(cs)
        rec["D_loc"] = [str(v) for v in D]
        out["cases"].append(rec)
    with open(os.path.join(HERE, "schur_loc_golden.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
