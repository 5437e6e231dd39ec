"""Parameter studies of the smoother on the paper's benchmark problems.

Runs the stationary protocol of Sec. 4.1 (x <- x + K_hat^-1 (b - K x) with one
multigrid cycle as K_hat^-1, from x = 0; rate q = (r_j / r_{j-3})^(1/3)) on
synthetic meshes of the sizes the paper uses, and prints markdown tables:

  diagonals  q for the Schur-diagonal choices D~_S (exact, d, p, loc) against
             the number of smoothing steps m, Chebyshev degrees k_A = k_S = k
             in {0, 3} (the comparisons of the laser and cavity examples on
             2467 DoFs in 2D, 2312 DoFs in 3D);
  degrees    q and the reduction per second, -log10(q) / T_iter, over the
             Chebyshev degrees (k_A, k_S) and m with D~_S_d (148 739 DoFs in
             2D, 112 724 DoFs in 3D);
  cycles     V- against W-cycle for the same grid.

Problems (Sec. 4): `laser`, the unit square with mu = 0.0022, homogeneous
Dirichlet data and the Gaussian force f = (0, c1 exp(-c2 |x - x0|^2)),
x0 = (0.75, 0.75), c1 = 1e-3, c2 = 100; `cavity2d` / `cavity3d`, mu = 1,
f = 0, tangential unit velocity along x on the open top face (its edges
belong to the fixed walls), lifted into the right-hand side.

Usage: python -m paper_2205_15770_amd.sweep --case cavity2d --study degrees
Every number comes from the library's kernels; this module only sets up the
problems and formats the results.
"""
import argparse
import math
import sys
import time

import numpy as np

from . import StokesMG, SMG_BLOCK_MASS

CASES = {
    # coarse mesh, levels of the small (diagonals) and large (degrees) problem
    "laser": dict(dim=2, mu=0.0022, n_coarse=(4, 4), small_levels=3, large_levels=6),
    "cavity2d": dict(dim=2, mu=1.0, n_coarse=(4, 4), small_levels=3, large_levels=6),
    "cavity3d": dict(dim=3, mu=1.0, n_coarse=(2, 2, 2), small_levels=2, large_levels=4),
}


def _rhs(mg, case):
    """b of the case on the finest level, and the Dirichlet data (or None)."""
    import torch
    L = mg.n_levels - 1
    nu, np_ = mg.sizes(L)
    b = torch.zeros(nu + np_, dtype=torch.float64, device="cuda")
    X = mg.node_coordinates(L)
    d = X.shape[1]
    if case == "laser":
        f = np.zeros((d, X.shape[0]))
        f[1] = 1e-3 * np.exp(-100.0 * ((X[:, 0] - 0.75) ** 2 + (X[:, 1] - 0.75) ** 2))
        mg.apply_block(L, SMG_BLOCK_MASS, torch.tensor(f.ravel(), device="cuda"), b[:nu])
        return b, None
    # lid: x-velocity 1 on the top face, edges of that face excluded
    top = np.isclose(X[:, d - 1], 1.0)
    inner = np.ones(X.shape[0], dtype=bool)
    for a in range(d - 1):
        inner &= (X[:, a] > 1e-12) & (X[:, a] < 1.0 - 1e-12)
    ud = np.zeros((d, X.shape[0]))
    ud[0, top & inner] = 1.0
    udg = torch.tensor(ud.ravel(), device="cuda")
    mg.lift_dirichlet(L, udg, b)
    return b, udg


def run_one(case, levels, k_A, k_S, m, schur="d", cycle=1, maxit=30, rtol=1e-10):
    """Stationary protocol for one configuration: dict(q, iterations, t_iter_ms, dofs)."""
    import torch
    c = CASES[case]
    mg = StokesMG(dim=c["dim"], fe_degree=2, n_coarse=c["n_coarse"], n_levels=levels, mu=c["mu"],
                  cheb_deg_A=k_A, cheb_deg_S=k_S, smooth_steps=m, cycle_index=cycle, schur_diag=schur)
    try:
        L = levels - 1
        b, _ = _rhs(mg, case)
        x = torch.zeros_like(b)
        mg.solve_stationary(x, b, rtol=rtol, maxit=3)          # warm-up (first-launch costs)
        x.zero_()
        info = mg.solve_stationary(x, b, rtol=rtol, maxit=maxit)
        its = max(info["iterations"], 1)
        q = info["rate_q"]
        if info["status"] != 0 and not (info["rel_residual"] < 1.0):
            q = float("inf")
        res = dict(q=q, iterations=info["iterations"], t_iter_ms=info["t_solve_ms"] / its, dofs=mg.n_total(L))
        print(f"# {case} levels={levels} (k_A,k_S,m)=({k_A},{k_S},{m}) schur={schur} cycle={cycle}: "
              f"q={q:.4f} its={res['iterations']} t_iter={res['t_iter_ms']:.3f} ms", file=sys.stderr, flush=True)
        return res
    finally:
        mg.close()


def _fmt_q(q):
    return "—" if not (q < 1.0) else f"{q:.3f}"


def study_diagonals(case, out, ms=range(1, 9)):
    c = CASES[case]
    rows = []
    dofs = None
    for k in (0, 3):
        for schur in ("exact", "d", "p", "loc"):
            qs = []
            for m in ms:
                r = run_one(case, c["small_levels"], k, k, m, schur=schur)
                dofs = r["dofs"]
                qs.append(_fmt_q(r["q"]))
            rows.append(f"| {k} | {schur} | " + " | ".join(qs) + " |")
    out.write(f"\n### {case}: rate q by Schur diagonal, k_A = k_S = k ({dofs} DoFs, V-cycle)\n\n")
    out.write("| k | D~_S | " + " | ".join(f"m={m}" for m in ms) + " |\n")
    out.write("|---|---|" + "---|" * len(ms) + "\n")
    out.write("\n".join(rows) + "\n")


def study_degrees(case, out, cycle=1, ms=(1, 2, 3)):
    c = CASES[case]
    lines_q, lines_r = [], []
    dofs = None
    best = (0.0, None)
    for kA in range(4):
        for kS in range(4):
            cq, cr = [], []
            for m in ms:
                r = run_one(case, c["large_levels"], kA, kS, m, cycle=cycle)
                dofs = r["dofs"]
                q = r["q"]
                cq.append(_fmt_q(q))
                if q < 1.0 and q > 0.0:
                    red = -math.log10(q) / (r["t_iter_ms"] * 1e-3)
                    cr.append(f"{red:.0f}")
                    if red > best[0]:
                        best = (red, (kA, kS, m))
                else:
                    cr.append("—")
            lines_q.append(f"| ({kA},{kS}) | " + " | ".join(cq) + " |")
            lines_r.append(f"| ({kA},{kS}) | " + " | ".join(cr) + " |")
    name = "V" if cycle == 1 else "W"
    head = "| (k_A,k_S) | " + " | ".join(f"m={m}" for m in ms) + " |\n|---|" + "---|" * len(ms) + "\n"
    out.write(f"\n### {case}: rate q, {name}-cycle, D~_S_d ({dofs} DoFs)\n\n" + head + "\n".join(lines_q) + "\n")
    out.write(f"\n### {case}: reduction per second -log10(q)/T_iter [orders/s], {name}-cycle ({dofs} DoFs)\n\n"
              + head + "\n".join(lines_r) + "\n")
    if best[1] is not None:
        out.write(f"\nLargest reduction per second: (k_A,k_S,m) = {best[1]}, {best[0]:.0f} orders/s.\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--case", choices=list(CASES), required=True)
    ap.add_argument("--study", choices=["diagonals", "degrees", "cycles"], required=True)
    args = ap.parse_args(argv)
    out = sys.stdout
    t0 = time.perf_counter()
    if args.study == "diagonals":
        study_diagonals(args.case, out)
    elif args.study == "degrees":
        study_degrees(args.case, out, cycle=1)
    else:
        study_degrees(args.case, out, cycle=2)
    out.write(f"\n({time.perf_counter() - t0:.1f} s)\n")
    out.flush()


if __name__ == "__main__":
    main()
