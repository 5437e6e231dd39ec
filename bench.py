"""Benchmark of the matrix-free monolithic multigrid Stokes solver on one MI355X.

Workload (default): the 2D generalized Stokes problem, Q2-Q1 on a uniform
512 x 512 box mesh (2,364,419 DoFs), mu = rho = 1, gamma = 1e3, nodal body
force U[-1,1] per velocity DoF (seed 2), 7-level V-cycle with the inexact
symmetric Uzawa smoother (k_A, k_S, m) = (1, 1, 2).

A step is one solve K x = b to ||b - K x|| <= 1e-8 ||b|| from x = 0 by FP64
FGMRES(30) preconditioned with one FP32 V-cycle per iteration: every part of
the method (operator applications, Chebyshev-Jacobi Uzawa smoothing, residuals,
transfers, coarse solve, cycle, outer loop) runs in each step; the diagonals
and Chebyshev bounds are set up once before the timed region.  Each step ends
with sixteen finest-level velocity updates u_hat = u + A_hat^-1 (f - A u -
B^T p), A_hat^-1 = sigma Cheb(A, D_A, 1), in FP32 (one fused launch each: the
operator kernel that dominates the cycle) back to back between one pair of HIP
events on the solver's stream, on vector sets rotating through more memory
than the Infinity Cache holds: the roofline entry's duration.

value = DoFs solved per second: N * steps / (sum of the solve times of the
timed steps; each solve call returns synchronised), GDoF/s; the roofline
launches are timed separately (timed_region_ms_per_step holds both).  The
same line reports the vmult throughput (GDoF/s, FP64 and FP32, HBM-resident
vectors), the FP64-preconditioned solve, the 3D Q2-Q1 64^3 solve in both
precisions with its error against the oracle on the 16^3 mesh, and the CPU
oracle on a bounded sample (one thread and all host threads).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256e6          # Infinity Cache (MALL) capacity
# MI355X FP32 vector peak (256 CUs x 4 SIMDs x 2.4 GHz, packed issue); the
# kernels are built without packed FP32, which halves what they can issue
FP32_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "stokes2d_q2q1_512": dict(dim=2, fe_degree=2, n_coarse=(8, 8), n_levels=7, mu=1.0, rho=1.0, gamma=1e3,
                              desc="2D generalized Stokes Q2-Q1, 512x512 cells, 7 levels, gamma=1e3"),
    "stokes3d_q2q1_64": dict(dim=3, fe_degree=2, n_coarse=(2, 2, 2), n_levels=6, mu=1.0, rho=1.0, gamma=0.0,
                             force="manufactured", desc="3D Stokes Q2-Q1, 64^3 cells, 6 levels, manufactured f"),
    "stokes3d_q3q2_32_pert": dict(dim=3, fe_degree=3, n_coarse=(2, 2, 2), n_levels=5, mu=1.0, rho=1.0, gamma=0.0,
                                  force="manufactured", perturb=(0.2, 4), log_mu=(1.0, 100.0, 5),
                                  desc="3D Stokes Q3-Q2, 32^3 trilinear cells (interior vertices moved by "
                                       "<= 0.2 h, seed 4), mu = exp(8 Fourier modes) in [1, 100] (seed 5), "
                                       "5 levels, manufactured f"),
}


def synth_uniform(n, seed):
    import synth_inputs as si
    return si.uniform(n, seed)


def cells(wl):
    n = [c * 2 ** (wl["n_levels"] - 1) for c in wl["n_coarse"]]
    return (n + [1, 1])[:3]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="stokes2d_q2q1_512", choices=sorted(WORKLOADS) + ["batch2d_q2q1_64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--adjoint-check", type=int, default=0, metavar="NDIR",
                    help="also time the differentiable solve (forward + adjoint backward of "
                         "J = ||u - u_target||^2) and compare NDIR directional derivatives with "
                         "central differences (step 1e-5, solves to 1e-11)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 512 MiB device copy (scale reference for HBM counters)")
    return ap.parse_args()


def rhs(mg, level, dim, seed=2, force="random"):
    """b = [M_v f, 0] for a nodal force f (the library's mass kernel): random
    U[-1,1] per velocity DoF, or the nodal interpolant of the manufactured f."""
    import torch
    import synth_inputs as si
    nu, np_ = mg.sizes(level)
    if force == "manufactured":
        fn = si.manufactured_f(mg.node_coordinates(level), 1.0, 0.0, 1.0).T
    else:
        fn = si.nodal_random_f(dim, nu // dim, seed=seed)
    f = torch.tensor(fn.ravel(), dtype=torch.float64, device="cuda")
    b = torch.zeros(nu + np_, dtype=torch.float64, device="cuda")
    from paper_2205_15770_amd import SMG_BLOCK_MASS
    mg.apply_block(level, SMG_BLOCK_MASS, f, b[:nu])
    return b


# Plain sum-factorisation flops per DoF of K x (velocity passes, pressure
# passes, quadrature-point physics; counted per cell and divided by the DoFs
# per cell) for the 3D workloads, against which the vmult is vector-ALU bound.
FLOPS_PER_DOF = {"stokes3d_q2q1_64": 277.0, "stokes3d_q3q2_32_pert": 443.0}
FP64_PEAK_TFLOPS = 78.6


def time_vmult(mg, level, dtype, reps=10, max_pairs=None, flops_per_dof=None):
    """GDoF/s of y = K x, HIP events on the stream, rotating over as many
    (x, y) pairs as it takes to exceed twice the 256 MB Infinity Cache for the
    vector type (so x comes from HBM and y goes to it; max_pairs caps that for
    small levels, which then stay cache-resident); also the same launches on
    one pair (cache-resident) for comparison.  With flops_per_dof, also the
    achieved vector rate against the FP64 / FP32 vector peak."""
    import torch
    import synth_inputs as si
    n = mg.n_total(level)
    esize = 8 if dtype == torch.float64 else 4
    pairs = max(4, -(-int(2 * MALL_BYTES) // (2 * esize * n)))
    if max_pairs is not None:
        pairs = min(pairs, max_pairs)
    x0 = torch.tensor(si.uniform(n, 200), dtype=dtype, device="cuda")
    xs = [x0 * (1.0 + 0.01 * i) for i in range(pairs)]
    ys = [torch.empty(n, dtype=dtype, device="cuda") for _ in range(pairs)]
    for i in range(pairs):
        mg.vmult(level, xs[i], ys[i])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        for i in range(pairs):
            mg.vmult(level, xs[i], ys[i])
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / (reps * pairs)
    e0.record()
    for _ in range(reps * 4):
        mg.vmult(level, xs[0], ys[0])
    e1.record()
    torch.cuda.synchronize()
    t_hot = e0.elapsed_time(e1) * 1e-3 / (reps * 4)
    del xs, ys
    out = {"gdofs": round(n / t / 1e9, 2), "us": round(t * 1e6, 2),
           "hbm_gbs": round(2 * esize * n / t / 1e9, 1),
           "frac_of_hbm_peak": round(2 * esize * n / t / 1e9 / HBM_PEAK_GBS, 3),
           "pairs_rotated": pairs, "rotated_mb": round(2 * esize * n * pairs / 1e6, 1),
           "us_one_pair_cache_resident": round(t_hot * 1e6, 2),
           "gdofs_one_pair_cache_resident": round(n / t_hot / 1e9, 2)}
    if flops_per_dof is not None:
        peak = FP64_PEAK_TFLOPS if esize == 8 else FP32_PEAK_TFLOPS
        tfl = n * flops_per_dof / t / 1e12
        out["alu"] = {"flops_per_dof": flops_per_dof, "achieved_tflops": round(tfl, 2), "peak_tflops": peak,
                      "frac": round(tfl / peak, 3)}
    return out


def traffic_from_profiles(kernel_key):
    """Per-launch HBM bytes of `kernel_key` from the committed counter summary,
    if it was taken on the current kernel sources (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2205_15770_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2205_15770_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if rec.get("sources_sha256") != h.hexdigest():
        return None
    k = rec.get("kernels", {}).get(kernel_key)
    return None if k is None else k.get("bytes_per_launch")


def adjoint_check(wl, common, b, ndir):
    """Forward + adjoint backward of J = ||u - u_target||^2 (u_target the nodal
    interpolant of a seeded smooth random field, seed 6), gradients with
    respect to the per-cell log-viscosity and the nodal force; NDIR central
    differences of J along random directions of both.  FGMRES stagnates near
    1e-12 on this problem (cond(K) with mu spanning [1, 100]), so the solves
    go to 1e-11 and the step is 1e-5 (truncation error ~1e-10 relative)."""
    import numpy as np
    import torch
    import synth_inputs as si
    from paper_2205_15770_amd import StokesMG, SMG_BLOCK_MASS
    from paper_2205_15770_amd.adjoint import solve
    prob = {k: v for k, v in common.items() if k != "mu_cell"}
    prob["precision"] = "f64"
    L = wl["n_levels"] - 1
    mg = StokesMG(**common)
    X = mg.node_coordinates(L)
    nu, _ = mg.sizes(L)
    mg.close()
    ut = torch.tensor(si.smooth_random_field(X, seed=6).T.ravel(), dtype=torch.float64, device="cuda")
    fn = si.manufactured_f(X, 1.0, 0.0, 1.0).T.ravel()
    f0 = torch.tensor(fn, dtype=torch.float64, device="cuda")
    mu = common.get("mu_cell")
    ncell = int(np.prod(cells(wl)[:wl["dim"]]))
    lm0 = torch.tensor(np.log(mu) if mu is not None else np.zeros(ncell), dtype=torch.float64, device="cuda")

    def J(f, lm, rtol):
        x = solve(f, lm, rtol=rtol, maxit=500, **prob)
        return ((x[:nu] - ut) ** 2).sum()

    f = f0.clone().requires_grad_(True)
    lm = lm0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = J(f, lm, 1e-11)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rng = np.random.default_rng(20)
    h = 1e-5
    errs = []
    for _ in range(ndir):
        dl = torch.tensor(rng.standard_normal(ncell), dtype=torch.float64, device="cuda")
        df = torch.tensor(rng.standard_normal(nu), dtype=torch.float64, device="cuda")
        with torch.no_grad():
            fd = (J(f0 + h * df, lm0 + h * dl, 1e-11) - J(f0 - h * df, lm0 - h * dl, 1e-11)).item() / (2 * h)
        an = (lm.grad @ dl + f.grad @ df).item()
        errs.append(abs(fd - an) / max(abs(an), 1e-300))
    return {"J": loss.item(), "forward_s_incl_setup": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
            "fd_directions": ndir, "fd_step": h, "fd_rel_err_max": max(errs) if errs else None,
            "fd_rel_err_median": float(np.median(errs)) if errs else None}


def bench_batch(args):
    """64 independent 2D generalized Stokes Q2-Q1 problems (side counts
    log-uniform in [32, 512] snapped to c 2^j, c in 4..7, seed 7; gamma ~
    U[0, 1e4]; nodal random f, seed 8 + i), solved together to 1e-8 by
    smg_batch_solve: every stage of the cycle and of the Krylov iteration is
    one packed launch over all problems, the batched cycle one graph launch,
    the kernel variants chosen by smg_batch_autotune; FP32-mixed and FP64
    cycles.  value = total DoFs solved per second."""
    import numpy as np
    import torch
    import synth_inputs as si
    from paper_2205_15770_amd import StokesBatch, SMG_BLOCK_MASS
    inst = si.batch_instances()
    out = {}
    for prec in ("f32", "f64"):
        probs = [dict(dim=2, fe_degree=2, n_coarse=(d["c"], d["c"]), n_levels=d["levels"], mu=1.0, rho=1.0,
                      gamma=d["gamma"], cheb_deg_A=1, cheb_deg_S=1, smooth_steps=2, cycle_index=1, schur_diag="d",
                      precision=prec) for d in inst]
        t0 = time.perf_counter()
        batch = StokesBatch(probs)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        xs, bs = [], []
        for i, mg in enumerate(batch.solvers):
            L = mg.n_levels - 1
            nu, np_ = mg.sizes(L)
            f = torch.tensor(si.nodal_random_f(2, nu // 2, seed=8 + i).ravel(), dtype=torch.float64, device="cuda")
            b = torch.zeros(nu + np_, dtype=torch.float64, device="cuda")
            mg.apply_block(L, SMG_BLOCK_MASS, f, b[:nu])
            bs.append(b)
            xs.append(torch.zeros(nu + np_, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        ntot = sum(mg.n_total(mg.n_levels - 1) for mg in batch.solvers)
        best, tune = batch.autotune(probe_cycles=5)
        launches, _ = batch.info()
        print(f"# batch {prec}: setup {t_setup:.2f} s, N = {ntot}, variant {best} {tune}, "
              f"{launches} packed launches per cycle", file=sys.stderr, flush=True)
        for _ in range(max(args.warmup, 1)):
            for x in xs:
                x.zero_()
            batch.solve(xs, bs, rtol=1e-8, maxit=300)
        times, infos = [], None
        for _ in range(args.steps):
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = batch.solve(xs, bs, rtol=1e-8, maxit=300)
            times.append(time.perf_counter() - t0)
        its = np.array([i["iterations"] for i in infos])
        wall = float(np.median(times))
        out[prec] = {"wall_ms": round(wall * 1e3, 2), "gdofs": round(ntot / wall / 1e9, 4), "variant": best,
                     "autotune_ms_per_cycle": [round(t, 3) for t in tune],
                     "packed_launches_per_cycle": launches, "graph_launches_per_cycle": 1,
                     "iterations_min_max": [int(its.min()), int(its.max())],
                     "max_rel_residual": max(i["rel_residual"] for i in infos), "setup_s": round(t_setup, 2)}
        batch.close()
        torch.cuda.synchronize()
    res = {"metric": "GDoF/s Stokes vmult; solve time to 1e-8 resid, FP32-mixed vs FP64",
           "value": out["f32"]["gdofs"], "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": out["f32"]["wall_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 cycle / f64 outer", "data": "synthetic",
           "config": {"workload": "batch2d_q2q1_64", "instances": len(inst), "dofs": ntot,
                      "description": "64 2D generalized Stokes Q2-Q1 problems, n log-uniform in [32, 512], "
                                     "gamma ~ U[0, 1e4], solved together to 1e-8 (smg_batch_solve, packed launches)"},
           "batch": out, "speedup_mixed_vs_f64": round(out["f64"]["wall_ms"] / out["f32"]["wall_ms"], 3)}
    print(json.dumps(res))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_solve_timed(ora, asm, b, threads):
    """The oracle's FGMRES(30) + FP64 V-cycle solve to 1e-8 and 20 CSR SpMVs
    of K, with the BLAS/OpenMP pools limited to `threads` (None = as the
    process starts them); returns wall times and the CPU time / wall time
    ratio (threads actually busy on average)."""
    from threadpoolctl import threadpool_limits
    import synth_inputs as si
    from oracle.krylov import fgmres
    ctx = threadpool_limits(threads) if threads else None
    try:
        c0, t0 = time.process_time(), time.perf_counter()
        x, hist = fgmres(asm.K, ora.precondition, b, rtol=1e-8)
        t = time.perf_counter() - t0
        busy = (time.process_time() - c0) / t
        xv = si.uniform(asm.K.shape[0], 1)
        t1 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            asm.K @ xv
        tv = (time.perf_counter() - t1) / reps
    finally:
        if ctx is not None:
            ctx.unregister()
    return x, hist, t, tv, busy


def cpu_baseline():
    """The oracle (assembled CSR, FP64, the same smoother, cycle and FGMRES;
    plain NumPy/SciPy as it stands) on a bounded sample of the workload: the
    same generalized Stokes problem on a 256 x 256 mesh (6 levels), timed
    with one thread and with every host thread; setup (assembly) excluded
    and reported.  Also the library's solves of that system against the
    oracle's solution."""
    import numpy as np
    import synth_inputs as si
    from oracle.mesh import make_hierarchy
    from oracle.mg import Multigrid, pressure_mean_free
    t0 = time.perf_counter()
    meshes = make_hierarchy(2, (8, 8), 6, 2)
    ora = Multigrid(meshes, mu=1.0, gamma=1e3, rho=1.0, k_A=1, k_S=1, smooth_steps=2)
    t_asm = time.perf_counter() - t0
    asm = ora.levels[-1]
    b = asm.rhs_from_nodal_f(si.nodal_random_f(2, meshes[-1].n_vnode, seed=2))
    n = asm.K.shape[0]
    x, hist, t1c, tv1, busy1 = _oracle_solve_timed(ora, asm, b, 1)
    _, _, tall, tvall, busyall = _oracle_solve_timed(ora, asm, b, None)
    # the library's solves of the same system (FP32 and FP64 V-cycle) against
    # the oracle's solution, pressure means removed from both
    import torch
    from paper_2205_15770_amd import StokesMG
    xo = pressure_mean_free(asm, x)
    diffs = {}
    for prec in ("f32", "f64"):
        mg = StokesMG(dim=2, fe_degree=2, n_coarse=(8, 8), n_levels=6, mu=1.0, rho=1.0, gamma=1e3, cheb_deg_A=1,
                      cheb_deg_S=1, smooth_steps=2, cycle_index=1, schur_diag="d", precision=prec)
        bg = torch.tensor(b, dtype=torch.float64, device="cuda")
        xg = torch.zeros_like(bg)
        mg.solve(xg, bg, rtol=1e-8, maxit=300)
        xs = pressure_mean_free(asm, xg.cpu().numpy())
        diffs["f32_mixed" if prec == "f32" else "f64"] = float(np.linalg.norm(xs - xo) / np.linalg.norm(xo))
        mg.close()
    nproc = os.cpu_count()
    return {"value": n / t1c / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FGMRES(30) + FP64 V-cycle solve to 1e-8 of the same generalized Stokes problem on "
                      f"256x256 cells ({n} DoFs, 6 levels), {len(hist) - 1} iterations, {t1c:.2f} s on one thread, "
                      f"assembly {t_asm:.1f} s excluded",
            "cpu_model": _cpu_model(), "nproc": nproc,
            "one_thread": {"solve_s": round(t1c, 3), "gdofs": n / t1c / 1e9, "spmv_gdofs": n / tv1 / 1e9,
                           "busy_threads": round(busy1, 2)},
            "all_threads": {"threads_allowed": nproc, "solve_s": round(tall, 3), "gdofs": n / tall / 1e9,
                            "spmv_gdofs": n / tvall / 1e9, "busy_threads": round(busyall, 2),
                            "note": "SciPy's CSR kernels run on one thread; only BLAS calls can use more"},
            "assembly_s": round(t_asm, 2),
            "library_vs_oracle_solution_rel_diff": diffs}


def c3_block(steps):
    """The 3D Stokes Q2-Q1 workload on 64^3 cells (6,714,692 DoFs, 6 levels,
    mu = 1, gamma = 0, the nodal interpolant of the manufactured force):
    FGMRES(30) to 1e-8 with the FP32 and the FP64 V-cycle (setup excluded,
    reported), the vmult rates in both precisions over more vector pairs than
    the Infinity Cache holds, and the error of the library's solves against
    the FP64 oracle on the 16^3 mesh of the same problem (112,724 DoFs, 4
    levels; the 3D driven-cavity size of the paper's Sec. 4.5), the oracle
    solved to 1e-12."""
    import numpy as np
    import torch
    from paper_2205_15770_amd import StokesMG
    wl = WORKLOADS["stokes3d_q2q1_64"]
    common = dict(dim=3, fe_degree=2, n_coarse=wl["n_coarse"], n_levels=wl["n_levels"], mu=1.0, rho=1.0,
                  gamma=0.0, cheb_deg_A=1, cheb_deg_S=1, smooth_steps=2, cycle_index=1, schur_diag="d")
    L = wl["n_levels"] - 1
    out = {"workload": "stokes3d_q2q1_64", "description": wl["desc"]}
    sols = {}
    for prec in ("f32", "f64"):
        t0 = time.perf_counter()
        mg = StokesMG(precision=prec, **common)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        N = mg.n_total(L)
        b = rhs(mg, L, 3, force="manufactured")
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        mg.solve(x, b, rtol=1e-8, maxit=300)
        tt, info = [], None
        for _ in range(steps):
            x.zero_()
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            info = mg.solve(x, b, rtol=1e-8, maxit=300)
            tt.append(time.perf_counter() - s0)
        sols[prec] = x
        key = "f32_mixed" if prec == "f32" else "f64"
        out[key] = {"solve_ms_median": round(float(np.median(tt)) * 1e3, 2),
                    "solve_ms_min": round(min(tt) * 1e3, 2), "iterations": info["iterations"],
                    "rel_residual": info["rel_residual"], "setup_s": round(t_setup, 2),
                    "gdofs_solved": round(N / float(np.median(tt)) / 1e9, 4)}
        if prec == "f32":
            out["dofs"] = N
            out["vmult_f64"] = time_vmult(mg, L, torch.float64, flops_per_dof=FLOPS_PER_DOF["stokes3d_q2q1_64"])
            out["vmult_f32"] = time_vmult(mg, L, torch.float32, flops_per_dof=FLOPS_PER_DOF["stokes3d_q2q1_64"])
        mg.close()
        torch.cuda.synchronize()
    out["speedup_mixed_vs_f64"] = round(out["f64"]["solve_ms_median"] / out["f32_mixed"]["solve_ms_median"], 3)
    out["rel_diff_mixed_vs_f64_solution"] = (torch.linalg.norm(sols["f32"] - sols["f64"]) /
                                             torch.linalg.norm(sols["f64"])).item()
    del sols
    # error against the FP64 oracle on the 16^3 mesh
    from oracle.mesh import make_hierarchy
    from oracle.mg import Multigrid, pressure_mean_free
    from oracle.krylov import fgmres
    import synth_inputs as si
    meshes = make_hierarchy(3, (2, 2, 2), 4, 2)
    ora = Multigrid(meshes, mu=1.0, gamma=0.0, rho=1.0, k_A=1, k_S=1, smooth_steps=2)
    asm = ora.levels[-1]
    X = meshes[-1].velocity_node_coordinates()
    bo = asm.rhs_from_nodal_f(si.manufactured_f(X, 1.0, 0.0, 1.0).T)
    xo, _ = fgmres(asm.K, ora.precondition, bo, rtol=1e-12)
    xo = pressure_mean_free(asm, xo)
    nu = asm.A.shape[0]
    err = {}
    for prec in ("f32", "f64"):
        mg = StokesMG(precision=prec, **dict(common, n_levels=4))
        bg = torch.tensor(bo, dtype=torch.float64, device="cuda")
        xg = torch.zeros_like(bg)
        info = mg.solve(xg, bg, rtol=1e-8, maxit=300)
        xs = pressure_mean_free(asm, xg.cpu().numpy())
        err["f32_mixed" if prec == "f32" else "f64"] = {
            "u_rel_err": float(np.linalg.norm(xs[:nu] - xo[:nu]) / np.linalg.norm(xo[:nu])),
            "p_rel_err": float(np.linalg.norm(xs[nu:] - xo[nu:]) / np.linalg.norm(xo[nu:])),
            "iterations": info["iterations"]}
        mg.close()
    out["vs_oracle_16cubed"] = dict(err, dofs=int(asm.K.shape[0]),
                                    note="library solves to 1e-8 against the oracle's FGMRES solve to 1e-12, "
                                         "pressure means removed")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (--gpus 1); "
                                   "multi-GPU sharding is described in DESIGN.md, not built"}))
        sys.exit(2)
    import torch
    from paper_2205_15770_amd import StokesMG
    torch.cuda.set_device(0)
    if args.workload == "batch2d_q2q1_64":
        bench_batch(args)
        return
    wl = WORKLOADS[args.workload]
    common = dict(dim=wl["dim"], fe_degree=wl["fe_degree"], n_coarse=wl["n_coarse"], n_levels=wl["n_levels"],
                  mu=wl["mu"], rho=wl["rho"], gamma=wl["gamma"], cheb_deg_A=1, cheb_deg_S=1, smooth_steps=2,
                  cycle_index=1, schur_diag="d")
    n_fine = cells(wl)[:wl["dim"]]
    if "perturb" in wl:
        import synth_inputs as si
        amp, seed = wl["perturb"]
        common["fine_vertices"] = si.perturbed_box_vertices(n_fine, dim=wl["dim"], amplitude=amp, seed=seed)
    if "log_mu" in wl:
        import synth_inputs as si
        lo, hi, seed = wl["log_mu"]
        common["mu_cell"] = si.fourier_log_viscosity(n_fine[0], dim=wl["dim"], mu_min=lo, mu_max=hi, seed=seed)
    L = wl["n_levels"] - 1
    t_setup0 = time.perf_counter()
    mg = StokesMG(precision="f32", **common)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup0
    N = mg.n_total(L)
    b = rhs(mg, L, wl["dim"], force=wl.get("force", "random"))
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    print(f"# setup {t_setup:.2f} s, N = {N}", file=sys.stderr, flush=True)
    # the dominant operator kernel of the cycle.  On 2D box levels that is the
    # fused velocity update of the Uzawa step (the residual f - A u - B^T p and
    # the first Chebyshev step of A_hat^-1 = sigma Cheb(A, D_A, 1) in one
    # launch, FP32), one launch per smg_velocity_update call; where that update
    # is more than one launch, the finest-level Chebyshev application of A,
    # one launch per smg_chebyshev call.  Inputs and outputs rotate over ROT
    # sets, more than the Infinity Cache holds, so every launch reads its
    # inputs from HBM and writes its output to it.
    nu, _ = mg.sizes(L)
    x1 = torch.tensor(synth_uniform(N, 31), dtype=torch.float32, device="cuda")
    b1 = torch.tensor(synth_uniform(N, 32), dtype=torch.float32, device="cuda")
    mg.profile(True)
    mg.velocity_update(L, x1, b1)
    probe = mg.profile_report()
    mg.profile(False)
    fused = len(probe) == 1
    if fused:
        key = next(iter(probe))
        set_bytes = 4 * (2 * N + nu)
    else:
        key = f"cheb_A/v3/blk1/f32/{'x'.join(str(v) for v in cells(wl))}"
        set_bytes = 2 * 4 * nu
    rot = max(8, -(-int(2 * MALL_BYTES) // set_bytes))
    if fused:
        ins = [(x1 * (1.0 + 0.01 * i), b1 * (1.0 - 0.01 * i)) for i in range(rot)]
        outs = [torch.empty(nu, dtype=torch.float32, device="cuda") for _ in range(rot)]

        def launch(i):
            mg.velocity_update(L, ins[i][0], ins[i][1], outs[i])
    else:
        ins = [x1[:nu] * (1.0 + 0.01 * i) for i in range(rot)]
        outs = [torch.empty(nu, dtype=torch.float32, device="cuda") for _ in range(rot)]

        def launch(i):
            mg.chebyshev(L, 0, ins[i], outs[i])
    del x1, b1
    per_step = 16
    for _ in range(args.warmup):
        x.zero_()
        mg.solve(x, b, rtol=1e-8, maxit=300)
        for i in range(rot):
            launch(i)
    print("# warmup done", file=sys.stderr, flush=True)
    # per step: the solve (host clock; it returns synchronised), then per_step
    # launches of the kernel back to back on per_step different vector sets,
    # between one pair of HIP events on the solver's stream (the stream the
    # library launches on): issue-to-issue time per launch, the inter-dispatch
    # gap included
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    solve_s = 0.0
    for s in range(args.steps):
        x.zero_()
        s0 = time.perf_counter()
        infos.append(mg.solve(x, b, rtol=1e-8, maxit=300))   # returns synchronised
        solve_s += time.perf_counter() - s0
        ev[s][0].record(stream)
        for j in range(per_step):
            launch((s * per_step + j) % rot)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("# timed steps done", file=sys.stderr, flush=True)
    elapsed = t1 - t0
    value = N * args.steps / solve_s / 1e9
    kern_ms_rot = sum(e0.elapsed_time(e1) for e0, e1 in ev) / (args.steps * per_step)
    # the same launch back to back on one set (cache-resident), for comparison
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    launch(0)
    e0.record(stream)
    for _ in range(16):
        launch(0)
    e1.record(stream)
    torch.cuda.synchronize()
    kern_hot_ms = e0.elapsed_time(e1) / 16
    # algorithmic bytes of exactly that launch (the library's own accounting
    # of the call: every vector the kernel reads or writes, once)
    mg.profile(True)
    launch(0)
    cnt1, _, nbytes1 = mg.profile_report()[key]
    mg.profile(False)
    bytes_per_launch = nbytes1 / cnt1
    # the plain Chebyshev application of A (the roofline kernel when the
    # update is not fused), rotated the same way, for comparison
    plain = None
    if fused:
        rs = [outs[i] for i in range(min(rot, 2 * per_step))]
        r_outs = [ins[i][0][:nu] for i in range(len(rs))]
        for i in range(len(rs)):
            mg.chebyshev(L, 0, rs[i], r_outs[i])
        e0.record(stream)
        for i in range(len(rs)):
            mg.chebyshev(L, 0, rs[i], r_outs[i])
        e1.record(stream)
        torch.cuda.synchronize()
        pk = f"cheb_A/v3/blk1/f32/{'x'.join(str(v) for v in cells(wl))}"
        mg.profile(True)
        mg.chebyshev(L, 0, rs[0], r_outs[0])
        pc, _, pb = mg.profile_report()[pk]
        mg.profile(False)
        p_ms = e0.elapsed_time(e1) / len(rs)
        plain = {"kernel": pk, "avg_us": round(p_ms * 1e3, 2),
                 "frac": round(pb / pc / (p_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "traffic": traffic_from_profiles(pk)}
        del rs, r_outs
    del ins, outs
    # per-kernel shares of one eager solve (kernel timing on), for the record
    mg.profile(True)
    x.zero_()
    mg.solve(x, b, rtol=1e-8, maxit=300)
    rep = mg.profile_report()
    mg.profile(False)
    kern_ms = sum(v[1] for v in rep.values())
    dom = max(rep, key=lambda k: rep[k][1])
    cnt, ms, nbytes = rep[key]
    achieved = bytes_per_launch / (kern_ms_rot * 1e-3) / 1e9
    traffic = traffic_from_profiles(key)
    # the same launch as vector-ALU work: the sum-factorised A of every cell
    # (2D: 4 passes of (k+1)^3 FMA per component, 3D: 7 passes of (k+1)^4;
    # the B^T p part of the fused residual is left out, so a lower bound),
    # against the FP32 vector peak (box cells only)
    alu = None
    if "perturb" not in wl:
        k, d = wl["fe_degree"], wl["dim"]
        ncell = 1
        for v in cells(wl)[:d]:
            ncell *= v
        fma = d * (4 * (k + 1) ** 3 if d == 2 else 7 * (k + 1) ** 4)
        flops = 2.0 * fma * ncell
        tfl = flops / (kern_ms_rot * 1e-3) / 1e12
        alu = {"achieved": round(tfl, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": round(tfl / FP32_PEAK_TFLOPS, 4), "flops_per_launch": flops}
    set_desc = "x (u, p), b (f, g) and u_hat" if fused else "r and out"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": key, "avg_us": round(kern_ms_rot * 1e3, 2),
                "avg_us_definition": f"{args.steps} x {per_step} launches in the timed steps, {per_step} back to back "
                                     f"per step between one HIP event pair (issue-to-issue time, inter-dispatch gap "
                                     f"included), {set_desc} rotating over {rot} vector sets "
                                     f"({set_bytes * rot / 1e6:.0f} MB, more than the 256 MB Infinity Cache)",
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "algorithmic_bytes_definition":
                    "u, p, f and D_A^-1 read, u_hat written, each once ((4 N_u + N_p) x 4 B)" if fused else
                    "r and D_A^-1 read, out written, each once (3 x 4 B x N_u)",
                "avg_us_one_pair_cache_resident": round(kern_hot_ms * 1e3, 2),
                "frac_one_pair_cache_resident": round(bytes_per_launch / (kern_hot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "launches_in_solve": cnt, "algorithmic_bytes_per_launch_in_solve": nbytes / cnt,
                "share_of_solve_kernel_time": round(ms / kern_ms, 3),
                "largest_kernel_in_solve": dom, "alu": alu, "plain_cheb_A_rotated": plain}
    extra = {}
    if not args.quick:
        fpd = FLOPS_PER_DOF.get(args.workload)
        extra["vmult"] = {"f64": time_vmult(mg, L, torch.float64, flops_per_dof=fpd),
                          "f32": time_vmult(mg, L, torch.float32, flops_per_dof=fpd)}
        # FP64 vmult on every level (levels below the finest rotate over at
        # most 64 vector pairs: from 128^2 down they stay in the Infinity Cache)
        extra["vmult_f64_levels_gdofs"] = {
            "x".join(str(v >> (L - l)) for v in cells(wl)[:wl["dim"]]): time_vmult(
                mg, l, torch.float64, reps=5, max_pairs=64)["gdofs"] for l in range(L + 1)}
        x_mixed = x.clone()
        mg64 = StokesMG(precision="f64", **common)
        x64 = torch.zeros_like(x)
        mg64.solve(x64, b, rtol=1e-8, maxit=300)
        tt = []
        for _ in range(2):
            x64.zero_()
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            i64 = mg64.solve(x64, b, rtol=1e-8, maxit=300)
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - s0)
        err = (torch.linalg.norm(x_mixed - x64) / torch.linalg.norm(x64)).item()
        extra["solve"] = {"f32_mixed_ms": round(solve_s / args.steps * 1e3, 3), "f64_ms": round(min(tt) * 1e3, 3),
                          "speedup_mixed_vs_f64": round(min(tt) / (solve_s / args.steps), 3),
                          "setup_s_f32": round(t_setup, 2),
                          "iterations_mixed": infos[-1]["iterations"], "iterations_f64": i64["iterations"],
                          "rel_residual_mixed": infos[-1]["rel_residual"], "rel_residual_f64": i64["rel_residual"],
                          "rel_diff_mixed_vs_f64_solution": err}
        mg64.close()
        del x_mixed, x64
        mg.close()
        torch.cuda.synchronize()
        if args.workload == "stokes2d_q2q1_512":
            extra["c3"] = c3_block(max(3, args.steps // 2))
            print("# 3D block done", file=sys.stderr, flush=True)
    if args.adjoint_check:
        extra["adjoint"] = adjoint_check(wl, common, b, args.adjoint_check)
    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
    out = {"metric": "GDoF/s Stokes vmult; solve time to 1e-8 resid, FP32-mixed vs FP64",
           "value": round(value, 4), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(solve_s / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 cycle / f64 outer", "data": "synthetic",
           "config": {"workload": args.workload, "description": wl["desc"], "dofs": N,
                      "smoother": "(k_A,k_S,m)=(1,1,2), D~_S_d, V-cycle", "rtol": 1e-8,
                      "value_definition": "DoFs solved to 1e-8 per second: N * steps / (sum of the steps' solve "
                                          "times, host clock around each synchronising solve call)",
                      "timed_region_ms_per_step": round(elapsed / args.steps * 1e3, 3)},
           "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
