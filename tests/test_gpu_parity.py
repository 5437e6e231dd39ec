"""GPU parity: every entry point of the HIP library (through the C ABI) against
the FP64 CPU oracle on the same seeded inputs.

Sizes: meshes the oracle assembles in seconds that still span several tiles
with ragged last tiles in every direction (2D wave tiles own 7 x 7 cells, or
5 x 5 / 3 x 3 in the two- and three-stage fused launches; 3D column sweeps
own 8 x 6 cell columns, cell blocks 3 x 3 x 3 cells, the matrix-core cell
kernel 16 x 8 columns).  Tolerances:
  * FP64 operator applications: relative 2-norm error <= 1e-12 (a few hundred
    roundings of O(1) terms per entry on random inputs), and componentwise
    max_i |y - y_o|_i / (|K| |x|)_i <= 1e-12 (1e-4 in FP32), which is not
    hidden by cancellation in K x;
  * FP64 iterations (Chebyshev, smoother, cycle): <= 1e-10 (the same linear
    maps composed; rounding differences grow by the iteration's norm);
  * FP32: <= 2e-5 relative (single-precision roundings, same count).
"""
import contextlib
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth_inputs as si
from oracle.mesh import make_hierarchy
from oracle.mg import Multigrid, pressure_mean_free
from oracle.smoother import LevelSmoother
from oracle.rows import sample_Kx, sample_abs_Kx

pytestmark = pytest.mark.gpu

CONFIGS = {
    "2d_k2": dict(dim=2, k=2, n_coarse=(5, 3), levels=4),
    "2d_k3": dict(dim=2, k=3, n_coarse=(3, 2), levels=4),
    "3d_k2": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3),
    # the same levels through the column-sweep kernel (by default levels of at
    # most 32 cells per direction take the one-cell-per-lane block kernel)
    "3d_k2_sweep": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3, env={"SMG_BLOCK3D_MAX_N": "0"}),
    # the column sweep's tiles own 8 x 6 columns: a level of 10 x 14 x 6 cells
    # leaves ragged last tiles in x and y (and two z chunks)
    "3d_k2_sweep_ragged": dict(dim=3, k=2, n_coarse=(5, 7, 3), levels=2, env={"SMG_BLOCK3D_MAX_N": "0"}),
    # levels of at most 16 cells per direction use one wave per output plane
    # of the cell block by default; the same levels with one wave per block:
    "3d_k2_cellblock": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3, env={"SMG_PLANE3D_MAX_N": "0"}),
    # small 2D levels take one wave per output field, fuse the producer of
    # each Chebyshev right-hand side with the first Chebyshev step, and (k_S
    # = 1) run the pressure part of an Uzawa step as two three-stage launches
    # by default; the same levels with one wave per tile for all fields and
    # separate launches:
    "2d_k2_plain": dict(dim=2, k=2, n_coarse=(5, 3), levels=4,
                        env={"SMG_SPLIT2D_MAX_N": "0", "SMG_FUSE2D_MAX_N": "0", "SMG_FUSE3_2D_MAX_N": "0"}),
    "2d_k3_plain": dict(dim=2, k=3, n_coarse=(3, 2), levels=4,
                        env={"SMG_SPLIT2D_MAX_N": "0", "SMG_FUSE2D_MAX_N": "0", "SMG_FUSE3_2D_MAX_N": "0"}),
    # large 2D levels run the fused producer + Chebyshev launches on
    # workgroups of several waves that exchange faces through LDS; the same
    # small meshes with that on every level (three-stage launches off, so that
    # every fused pair takes it), in its three shapes:
    "2d_k2_wgf": dict(dim=2, k=2, n_coarse=(5, 3), levels=4,
                      env={"SMG_WGF2D_MIN_N": "1", "SMG_FUSE3_2D_MAX_N": "0"}),
    "2d_k3_wgf": dict(dim=2, k=3, n_coarse=(3, 2), levels=4,
                      env={"SMG_WGF2D_MIN_N": "1", "SMG_FUSE3_2D_MAX_N": "0"}),
    "2d_k2_wgf22": dict(dim=2, k=2, n_coarse=(5, 3), levels=4,
                        env={"SMG_WGF2D_MIN_N": "1", "SMG_WGF2D_SHAPE": "22", "SMG_FUSE3_2D_MAX_N": "0"}),
    "2d_k3_wgf44": dict(dim=2, k=3, n_coarse=(3, 2), levels=4,
                        env={"SMG_WGF2D_MIN_N": "1", "SMG_WGF2D_SHAPE": "44", "SMG_FUSE3_2D_MAX_N": "0"}),
    # FP32 Chebyshev steps for A on the matrix-core cell kernel (by default
    # levels of at least 64 cells per direction) on every level: uniform
    # viscosity with gamma rho != 0 (one cell matrix), and per-cell viscosity
    # with gamma = 0 (the viscosity scales the cell input); ragged 17 x 9
    # column tiles in x and y
    "3d_k2_mfma": dict(dim=3, k=2, n_coarse=(5, 3, 2), levels=3, percell=False,
                       env={"SMG_MFMA3D_MIN_N": "1", "SMG_BLOCK3D_MAX_N": "0"}),
    "3d_k2_mfma_mucell": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3, gamma=0.0,
                              env={"SMG_MFMA3D_MIN_N": "1", "SMG_BLOCK3D_MAX_N": "0"}),
    "3d_k3": dict(dim=3, k=3, n_coarse=(2, 2, 3), levels=2),
    # vertex-given (multilinear) cells: interior vertices of the finest mesh
    # moved by up to 0.2 h, coarse levels take the finest vertices
    "2d_k2_pert": dict(dim=2, k=2, n_coarse=(3, 2), levels=3, pert=True),
    "2d_k3_pert": dict(dim=2, k=3, n_coarse=(2, 3), levels=2, pert=True),
    "3d_k2_pert": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=2, pert=True),
    "3d_k3_pert": dict(dim=3, k=3, n_coarse=(2, 2, 2), levels=2, pert=True),
    # 3D general cells run the line-layout cell kernel by default; the same
    # meshes through the kernel with one lane per quadrature point:
    "3d_k2_pert_points": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=2, pert=True, env={"SMG_GEN3_LINES": "0"}),
    "3d_k3_pert_points": dict(dim=3, k=3, n_coarse=(2, 2, 2), levels=2, pert=True, env={"SMG_GEN3_LINES": "0"}),
}
PHYS = dict(gamma=7.0, rho=0.5)
_cache = {}


def _setup(name, c_p=0.0, kA=1, kS=1, schur="d", m=2, cycle=1, percell=True):
    key = (name, c_p, kA, kS, schur, m, cycle, percell)
    if key in _cache:
        return _cache[key]
    from paper_2205_15770_amd import StokesMG
    cfg = CONFIGS[name]
    dim, k, L = cfg["dim"], cfg["k"], cfg["levels"]
    n_f = [c * 2 ** (L - 1) for c in cfg["n_coarse"]]
    percell = percell and cfg.get("percell", True)
    gamma = cfg.get("gamma", PHYS["gamma"])
    mu_cell = si.uniform(int(np.prod(n_f)), 17, 0.5, 3.0) if percell else None
    verts = _vertices(name)
    meshes = make_hierarchy(dim, cfg["n_coarse"], L, k, fine_mu=mu_cell, fine_vertices=verts)
    ora = Multigrid(meshes, mu=1.0, gamma=gamma, rho=PHYS["rho"], c_p=c_p, k_A=kA, k_S=kS,
                    schur=schur, smooth_steps=m, cycle_index=cycle)
    with _env(cfg):
        gpu = StokesMG(dim=dim, fe_degree=k, n_coarse=cfg["n_coarse"], n_levels=L, mu=1.0, mu_cell=mu_cell,
                       gamma=gamma, rho=PHYS["rho"], c_pressure=c_p, cheb_deg_A=kA, cheb_deg_S=kS,
                       smooth_steps=m, cycle_index=cycle, schur_diag=schur, fine_vertices=verts)
    _cache[key] = (ora, gpu)
    return ora, gpu


@contextlib.contextmanager
def _env(cfg):
    """Kernel-choice variables (read when a solver is set up) of a config."""
    env = cfg.get("env", {})
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        yield
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _vertices(name):
    cfg = CONFIGS[name]
    if not cfg.get("pert"):
        return None
    n_f = [c * 2 ** (cfg["levels"] - 1) for c in cfg["n_coarse"]]
    return si.perturbed_box_vertices(n_f, dim=cfg["dim"], amplitude=0.2, seed=21)


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    a = a.detach().cpu().numpy().astype(np.float64) if torch.is_tensor(a) else a
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _compwise(y, ref, scale):
    """max_i |y - ref|_i / scale_i with scale = |K| |x| (rows with scale 0
    must match exactly)."""
    y = y.detach().cpu().numpy().astype(np.float64) if torch.is_tensor(y) else np.asarray(y, dtype=np.float64)
    d = np.abs(y - ref)
    z = scale == 0
    assert not np.any(d[z] != 0)
    return float(np.max(d[~z] / scale[~z])) if np.any(~z) else 0.0


def _inject_betas(ora, gpu):
    for l in range(1, ora.L + 1):
        gpu.set_eigs(l, ora.smoothers[l].beta_A, ora.smoothers[l].beta_S)


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("c_p", [0.0, 0.3])
def test_vmult_fp64_every_level(name, c_p):
    ora, gpu = _setup(name, c_p=c_p)
    for l in range(ora.L + 1):
        K = ora.levels[l].K
        x = si.uniform(K.shape[0], 100 + l)
        y = gpu.vmult(l, _dev(x))
        err = _rel(y, K @ x)
        assert err < 1e-12, (name, l, err)
        cw = _compwise(y, K @ x, abs(K) @ np.abs(x))
        assert cw < 1e-12, (name, l, cw)


@pytest.mark.parametrize("name", list(CONFIGS))
def test_vmult_fp32(name):
    ora, gpu = _setup(name)
    l = ora.L
    x = si.uniform(ora.levels[l].K.shape[0], 5)
    y = gpu.vmult(l, _dev(x, torch.float32))
    x32 = x.astype(np.float32).astype(np.float64)
    K = ora.levels[l].K
    assert _rel(y, K @ x32) < 2e-5
    assert _compwise(y, K @ x32, abs(K) @ np.abs(x32)) < 1e-4


@pytest.mark.parametrize("name", list(CONFIGS))
def test_residual_and_blocks(name):
    from paper_2205_15770_amd import SMG_BLOCK_A, SMG_BLOCK_BT, SMG_BLOCK_B, SMG_BLOCK_MASS
    ora, gpu = _setup(name)
    l = ora.L
    asm = ora.levels[l]
    nu = asm.A.shape[0]
    x = si.uniform(asm.K.shape[0], 11)
    b = si.uniform(asm.K.shape[0], 12)
    r = gpu.residual(l, _dev(x), _dev(b))
    assert _rel(r, b - asm.K @ x) < 1e-12
    u, p = x[:nu], x[nu:]
    assert _rel(gpu.apply_block(l, SMG_BLOCK_A, _dev(u)), asm.A @ u) < 1e-12
    assert _rel(gpu.apply_block(l, SMG_BLOCK_BT, _dev(p)), asm.B.T @ p) < 1e-12
    assert _rel(gpu.apply_block(l, SMG_BLOCK_B, _dev(u)), asm.B @ u) < 1e-12
    # mass load vector of a nodal field, boundary values included
    d = ora.meshes[l].dim
    f = si.uniform(nu, 13).reshape(d, -1)
    ref = asm.rhs_from_nodal_f(f)[:nu]
    assert _rel(gpu.apply_block(l, SMG_BLOCK_MASS, _dev(f.ravel())), ref) < 1e-12


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("schur", ["d", "loc", "p", "exact"])
def test_diagonals(name, schur):
    ora, gpu = _setup(name, schur=schur, c_p=0.2)
    # the exact diagonal goes through A_hat^-1, whose Chebyshev coefficients
    # depend on each side's own Lanczos estimate of beta_A
    tol = 1e-10 if schur == "exact" else 1e-13
    for l in range(1, ora.L + 1):
        S = ora.smoothers[l]
        assert _rel(gpu.diagonal(l, 0), S.D_A) < 1e-13
        assert _rel(gpu.diagonal(l, 1), S.D_S) < tol


@pytest.mark.parametrize("name", list(CONFIGS))
def test_lanczos_bounds(name):
    ora, gpu = _setup(name)
    for l in range(1, ora.L + 1):
        bA, bS = gpu.eigs(l)
        assert abs(bA - ora.smoothers[l].beta_A) < 1e-8 * bA
        assert abs(bS - ora.smoothers[l].beta_S) < 1e-8 * bS


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("kA,kS", [(0, 0), (1, 1), (3, 2), (2, 1)])
def test_chebyshev_and_smoother(name, kA, kS):
    ora, gpu = _setup(name, kA=kA, kS=kS)
    _inject_betas(ora, gpu)
    l = ora.L
    S = ora.smoothers[l]
    nu = S.nu
    r = si.uniform(nu, 21) * ora.levels[l].free_u
    assert _rel(gpu.chebyshev(l, 0, _dev(r)), S.Ainv(r)) < 1e-10
    rp = si.uniform(ora.levels[l].B.shape[0], 22)
    assert _rel(gpu.chebyshev(l, 1, _dev(rp)), S.Sinv(rp)) < 1e-10
    n = ora.levels[l].K.shape[0]
    x = si.uniform(n, 23)
    b = si.uniform(n, 24)
    xg = _dev(x)
    gpu.smooth(l, xg, _dev(b), 2)
    assert _rel(xg, S.smooth(x, b, 2)) < 1e-10
    # FP32 smoother on the same data
    x32 = _dev(x, torch.float32)
    gpu.smooth(l, x32, _dev(b, torch.float32), 1)
    assert _rel(x32, S.smooth(x, b, 1)) < 1e-4


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("kA", [0, 1, 3])
def test_velocity_update(name, kA):
    """u_hat = u + A_hat^-1 (f - A u - B^T p), the first line of the Uzawa
    step (Sec. 1), against the oracle's assembled blocks; the 2D configs
    without the _plain suffix take the fused residual + Chebyshev launch."""
    ora, gpu = _setup(name, kA=kA)
    _inject_betas(ora, gpu)
    for l in (ora.L, 1):
        S = ora.smoothers[l]
        nu = S.nu
        n = ora.levels[l].K.shape[0]
        x = si.uniform(n, 25 + l)
        b = si.uniform(n, 26 + l)
        ref = x[:nu] + S.Ainv(b[:nu] - S.A @ x[:nu] - S.B.T @ x[nu:])
        assert _rel(gpu.velocity_update(l, _dev(x), _dev(b)), ref) < 1e-10
        out32 = gpu.velocity_update(l, _dev(x, torch.float32), _dev(b, torch.float32))
        assert out32.dtype == torch.float32
        assert _rel(out32, ref) < 1e-4


def test_velocity_update_rejects_aliasing():
    from paper_2205_15770_amd import _lib
    ora, gpu = _setup("2d_k2")
    n = ora.levels[ora.L].K.shape[0]
    nu = ora.smoothers[ora.L].nu
    x = _dev(si.uniform(n, 27))
    with pytest.raises(_lib.SmgError):
        gpu.velocity_update(ora.L, x, _dev(si.uniform(n, 28)), x[:nu])


@pytest.mark.parametrize("name", list(CONFIGS))
def test_transfers(name):
    ora, gpu = _setup(name)
    for l in range(1, ora.L + 1):
        P = ora.P[l]
        rf = si.uniform(P.shape[0], 30 + l)
        assert _rel(gpu.restrict(l, _dev(rf)), P.T @ rf) < 1e-13
        wc = si.uniform(P.shape[1], 40 + l)
        xf = si.uniform(P.shape[0], 50 + l)
        out = gpu.prolongate_add(l, _dev(wc), _dev(xf))
        assert _rel(out, xf + P @ wc) < 1e-13


@pytest.mark.parametrize("name", list(CONFIGS))
def test_coarse_solve(name):
    ora, gpu = _setup(name)
    a0 = ora.levels[0]
    b = si.uniform(a0.K.shape[0], 60)
    b[a0.constrained] = 0.0
    nu = a0.A.shape[0]
    b[nu:] -= b[nu:].mean()
    x = gpu.coarse_solve(_dev(b))
    assert _rel(x, ora.coarse_solve(b)) < 1e-11


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("cycle", [1, 2])
def test_cycle(name, cycle):
    ora, gpu = _setup(name, cycle=cycle)
    _inject_betas(ora, gpu)
    L = ora.L
    n = ora.levels[L].K.shape[0]
    f = si.nodal_random_f(ora.meshes[L].dim, ora.meshes[L].n_vnode, seed=2)
    b = ora.levels[L].rhs_from_nodal_f(f)
    x0 = si.uniform(n, 70) * 0.1
    x0[ora.levels[L].constrained] = 0.0
    xg = _dev(x0)
    gpu.vcycle(L, xg, _dev(b))
    assert _rel(xg, ora.cycle(L, x0.copy(), b)) < 1e-10
    # FP32 cycle
    x32 = _dev(x0, torch.float32)
    gpu.vcycle(L, x32, _dev(b, torch.float32))
    assert _rel(x32, ora.cycle(L, x0.copy(), b)) < 1e-4


@pytest.mark.parametrize("name", ["2d_k2", "2d_k3", "2d_k2_plain", "2d_k3_plain", "3d_k2"])
def test_uniform_viscosity(name):
    """Uniform viscosity (no per-cell field; the other parity tests give each
    cell its own mu): vmult on every level, the smoother and a V-cycle against
    the oracle, with C != 0."""
    ora, gpu = _setup(name, c_p=0.3, percell=False)
    _inject_betas(ora, gpu)
    for l in range(ora.L + 1):
        K = ora.levels[l].K
        x = si.uniform(K.shape[0], 200 + l)
        assert _rel(gpu.vmult(l, _dev(x)), K @ x) < 1e-12, l
        assert _rel(gpu.vmult(l, _dev(x, torch.float32)), K @ x.astype(np.float32).astype(np.float64)) < 2e-5, l
    L = ora.L
    S = ora.smoothers[L]
    n = ora.levels[L].K.shape[0]
    x = si.uniform(n, 223)
    b = si.uniform(n, 224)
    xg = _dev(x)
    gpu.smooth(L, xg, _dev(b), 2)
    assert _rel(xg, S.smooth(x, b, 2)) < 1e-10
    f = si.nodal_random_f(ora.meshes[L].dim, ora.meshes[L].n_vnode, seed=3)
    b = ora.levels[L].rhs_from_nodal_f(f)
    x0 = si.uniform(n, 71) * 0.1
    x0[ora.levels[L].constrained] = 0.0
    xg = _dev(x0)
    gpu.vcycle(L, xg, _dev(b))
    assert _rel(xg, ora.cycle(L, x0.copy(), b)) < 1e-10
    x32 = _dev(x0, torch.float32)
    gpu.vcycle(L, x32, _dev(b, torch.float32))
    assert _rel(x32, ora.cycle(L, x0.copy(), b)) < 1e-4


@pytest.mark.parametrize("name", ["2d_k2", "2d_k2_plain", "3d_k2", "3d_k2_sweep", "3d_k2_cellblock", "2d_k3", "3d_k3_pert"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fgmres_solve(name, precision):
    from paper_2205_15770_amd import StokesMG
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    ora, _ = _setup(name)
    cfg = CONFIGS[name]
    L = ora.L
    n_f = [c * 2 ** (cfg["levels"] - 1) for c in cfg["n_coarse"]]
    mu_cell = si.uniform(int(np.prod(n_f)), 17, 0.5, 3.0)
    with _env(cfg):
        gpu = StokesMG(dim=cfg["dim"], fe_degree=cfg["k"], n_coarse=cfg["n_coarse"], n_levels=cfg["levels"],
                       mu_cell=mu_cell, gamma=PHYS["gamma"], rho=PHYS["rho"], precision=precision,
                       fine_vertices=_vertices(name))
    asm = ora.levels[L]
    f = si.nodal_random_f(cfg["dim"], ora.meshes[L].n_vnode, seed=2)
    b = asm.rhs_from_nodal_f(f)
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    info = gpu.solve(x, _dev(b), rtol=1e-8, maxit=100)
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - asm.K @ xs) <= 1.05e-8 * np.linalg.norm(b)
    assert info["iterations"] < 40
    assert info["t_setup_ms"] > 0.0 and info["t_solve_ms"] > 0.0
    # against the oracle's direct solve (bordered, zero-mean pressure)
    nu = asm.A.shape[0]
    m = np.zeros(len(b))
    m[nu:] = asm.Mp @ np.ones(len(b) - nu)
    Kb = sp.bmat([[asm.K, sp.csr_matrix(m[:, None])], [sp.csr_matrix(m[None, :]), None]]).tocsc()
    xd = spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]
    # the error is bounded by cond(K) * rtol; these systems have cond ~ 1e3
    assert _rel(xs, xd) < 2e-5
    gpu.close()


@pytest.mark.parametrize("name", ["2d_k2", "3d_k2", "2d_k3_pert"])
def test_fgmres_solve_with_pressure_mass(name):
    """C = c_p M_p, c_p > 0: K is regular, the coarse solve inverts K_0
    without the zero-mean border and the solution is not shifted; the FGMRES
    solution against the oracle's sparse direct solve of K x = b."""
    from paper_2205_15770_amd import StokesMG
    import scipy.sparse.linalg as spla
    ora, _ = _setup(name, c_p=0.3)
    cfg = CONFIGS[name]
    L = ora.L
    n_f = [c * 2 ** (cfg["levels"] - 1) for c in cfg["n_coarse"]]
    mu_cell = si.uniform(int(np.prod(n_f)), 17, 0.5, 3.0)
    gpu = StokesMG(dim=cfg["dim"], fe_degree=cfg["k"], n_coarse=cfg["n_coarse"], n_levels=cfg["levels"],
                   mu_cell=mu_cell, gamma=PHYS["gamma"], rho=PHYS["rho"], c_pressure=0.3, precision="f32",
                   fine_vertices=_vertices(name))
    asm = ora.levels[L]
    b = asm.rhs_from_nodal_f(si.nodal_random_f(cfg["dim"], ora.meshes[L].n_vnode, seed=5))
    nu = asm.A.shape[0]
    b[nu:] = si.uniform(len(b) - nu, 6)            # a pressure right-hand side with non-zero mean
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    gpu.solve(x, _dev(b), rtol=1e-10, maxit=100)
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - asm.K @ xs) <= 1.05e-10 * np.linalg.norm(b)
    xd = spla.spsolve(asm.K.tocsc(), b)
    assert _rel(xs, xd) < 1e-6
    gpu.close()


def test_stationary_protocol_matches_oracle_rates():
    from oracle.krylov import stationary, rate_q
    ora, gpu = _setup("2d_k2", kA=3, kS=3, m=2)
    _inject_betas(ora, gpu)
    L = ora.L
    asm = ora.levels[L]
    X = ora.meshes[L].velocity_node_coordinates()
    b = asm.rhs_from_nodal_f(si.manufactured_f(X, 1.0, PHYS["gamma"], PHYS["rho"]).T)
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    info = gpu.solve_stationary(x, _dev(b), rtol=1e-10, maxit=15)
    xo, hist = stationary(asm.K, lambda x, b: ora.cycle(L, x, b), b, rtol=1e-10, maxit=15)
    h = np.array(hist) / hist[0]
    assert info["iterations"] == len(hist) - 1
    n = min(len(h), len(info["history"]))
    assert np.allclose(info["history"][:4], h[:4], rtol=1e-6)
    assert abs(info["rate_q"] - rate_q(hist)) < 0.05 * rate_q(hist) + 1e-3
    assert _rel(x, pressure_mean_free(asm, xo)) < 1e-8


@pytest.mark.parametrize("name", [n for n in CONFIGS if CONFIGS[n].get("pert")])
def test_node_coordinates_general_cells(name):
    ora, gpu = _setup(name)
    for l in range(ora.L + 1):
        X = gpu.node_coordinates(l)
        assert np.abs(X - ora.meshes[l].velocity_node_coordinates()).max() < 1e-14


def test_c1_protocol_16x16_stationary():
    """The 16^2 Q2-Q1 configuration with the paper's stationary protocol:
    3 levels, mu = 1, gamma = 0, manufactured f, (k_A, k_S, m) = (3, 3, 2),
    D~_S_d, V-cycle, to 1e-10 relative residual.  Residual history, rate q
    and solution against the oracle running the same iteration."""
    from paper_2205_15770_amd import StokesMG
    from oracle.krylov import stationary, rate_q
    meshes = make_hierarchy(2, (4, 4), 3, 2)
    ora = Multigrid(meshes, mu=1.0, gamma=0.0, rho=1.0, k_A=3, k_S=3, schur="d", smooth_steps=2, cycle_index=1)
    gpu = StokesMG(dim=2, fe_degree=2, n_coarse=(4, 4), n_levels=3, mu=1.0, gamma=0.0, rho=1.0,
                   cheb_deg_A=3, cheb_deg_S=3, smooth_steps=2, cycle_index=1, schur_diag="d")
    assert gpu.n_total(2) == 2467
    _inject_betas(ora, gpu)
    L = 2
    asm = ora.levels[L]
    X = meshes[L].velocity_node_coordinates()
    b = asm.rhs_from_nodal_f(si.manufactured_f(X, 1.0, 0.0, 1.0).T)
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    info = gpu.solve_stationary(x, _dev(b), rtol=1e-10, maxit=30)
    xo, hist = stationary(asm.K, lambda x, b: ora.cycle(L, x, b), b, rtol=1e-10, maxit=30)
    h = np.array(hist) / hist[0]
    assert info["iterations"] == len(hist) - 1
    # Both sides run the same iteration; their iterates differ by rounding,
    # so the computed relative residuals differ by up to about
    # eps * cond(K) (cond(K) ~ 1.1e5 here, on the complement of the constant
    # pressure) in absolute terms, besides 1e-6 relative: the early entries
    # agree to 1e-6, the late ones (~1e-10) to ~10 %.
    sv = np.linalg.svd(asm.K.toarray(), compute_uv=False)
    floor = np.finfo(np.float64).eps * sv[0] / sv[-2]
    hg = np.array(info["history"])
    assert np.all(np.abs(hg - h) <= 1e-6 * h + floor), (np.abs(hg - h) / h).max()
    # q = (h_j / h_{j-3})^(1/3): its rounding bound follows from the same floor
    j = len(h) - 1
    q = rate_q(hist)
    tol_q = 1e-6 * q + q * floor * (1.0 / h[j] + 1.0 / h[j - 3]) / 3.0
    assert abs(info["rate_q"] - q) <= tol_q, (info["rate_q"], q, tol_q)
    assert _rel(x, pressure_mean_free(asm, xo)) < 1e-8
    gpu.close()


@pytest.mark.parametrize("c_p", [0.2, 0.0])
@pytest.mark.parametrize("k,kA,kS", [(2, 1, 1), (2, 2, 1), (2, 3, 2), (2, 0, 1), (3, 1, 1), (3, 2, 1)])
def test_small_level_variants_equal_separate_launches(k, kA, kS, c_p):
    """The small-level 2D kernels (one wave per field; operator application
    fused with the first Chebyshev step; for k_S = 1 the pressure part of an
    Uzawa step in two three-stage launches) against the two-stage fusion
    alone and against one wave per tile with separate launches, on every
    level of the same problem: the same arithmetic in another launch order,
    so the results agree to rounding."""
    from paper_2205_15770_amd import StokesMG
    cfg = CONFIGS["2d_k2" if k == 2 else "2d_k3"]
    n_f = [c * 2 ** (cfg["levels"] - 1) for c in cfg["n_coarse"]]
    mu_cell = si.uniform(n_f[0] * n_f[1], 17, 0.5, 3.0)
    kw = dict(dim=2, fe_degree=k, n_coarse=cfg["n_coarse"], n_levels=cfg["levels"], mu_cell=mu_cell,
              gamma=PHYS["gamma"], rho=PHYS["rho"], c_pressure=c_p, cheb_deg_A=kA, cheb_deg_S=kS)
    a = StokesMG(**kw)
    with _env(CONFIGS["2d_k2_plain"]):
        b = StokesMG(**kw)
    with _env(dict(env={"SMG_FUSE3_2D_MAX_N": "0"})):
        c = StokesMG(**kw)
    for l in range(1, cfg["levels"]):
        bA, bS = a.eigs(l)
        b.set_eigs(l, bA, bS)
        c.set_eigs(l, bA, bS)
        n = a.n_total(l)
        for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
            x0 = _dev(si.uniform(n, 60 + l), dtype)
            rhs = _dev(si.uniform(n, 70 + l), dtype)
            xa, xb, xc = x0.clone(), x0.clone(), x0.clone()
            a.smooth(l, xa, rhs, 2)
            b.smooth(l, xb, rhs, 2)
            c.smooth(l, xc, rhs, 2)
            ref = xb.cpu().numpy().astype(np.float64)
            assert _rel(xa, ref) < tol, (l, dtype)
            assert _rel(xc, ref) < tol, (l, dtype)
    a.close()
    b.close()
    c.close()


def test_small_level_variants_full_size_hierarchy():
    """The three-stage launches on the 64^2 and 128^2 levels of the 512^2,
    7-level hierarchy (the largest levels they run on) against the two-stage
    fusion alone: smoothing steps agree to rounding."""
    from paper_2205_15770_amd import StokesMG
    kw = dict(dim=2, fe_degree=2, n_coarse=(8, 8), n_levels=7, gamma=1e3, rho=1.0)
    a = StokesMG(**kw)
    with _env(dict(env={"SMG_FUSE3_2D_MAX_N": "0"})):
        c = StokesMG(**kw)
    for l in (3, 4):
        bA, bS = a.eigs(l)
        c.set_eigs(l, bA, bS)
        n = a.n_total(l)
        for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
            x0 = _dev(si.uniform(n, 80 + l), dtype)
            rhs = _dev(si.uniform(n, 90 + l), dtype)
            xa, xc = x0.clone(), x0.clone()
            a.smooth(l, xa, rhs, 2)
            c.smooth(l, xc, rhs, 2)
            assert _rel(xa, xc.cpu().numpy().astype(np.float64)) < tol, (l, dtype)
    a.close()
    c.close()


def test_vmult_is_deterministic():
    ora, gpu = _setup("2d_k2")
    l = ora.L
    x = _dev(si.uniform(ora.levels[l].K.shape[0], 3))
    y1 = gpu.vmult(l, x).cpu().numpy()
    for _ in range(3):
        assert np.array_equal(gpu.vmult(l, x).cpu().numpy(), y1)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_full_size_2d_512_sampled_rows(dtype, tol):
    """The 512^2, 7-level generalized Stokes workload at full size: sampled rows
    of K x against the oracle's row-by-row definition, on the finest level (one
    wave per tile for all fields) and on the 128^2 level (one wave per tile
    and field)."""
    from paper_2205_15770_amd import StokesMG
    from oracle.mesh import BoxMesh
    gpu = StokesMG(dim=2, fe_degree=2, n_coarse=(8, 8), n_levels=7, gamma=1e3, rho=1.0)
    for L, nc in ((6, 512), (4, 128)):
        n = gpu.n_total(L)
        x = si.uniform(n, 99 + L)
        y = gpu.vmult(L, _dev(x, dtype)).cpu().numpy().astype(np.float64)
        mesh = BoxMesh(2, (nc, nc), 2)
        vd = 2 * nc + 1
        rng = np.random.default_rng(5)
        dofs = np.unique(np.concatenate([rng.integers(0, n, 400), np.arange(0, 40), np.arange(n - 40, n),
                                         [vd * 30 + 30, vd * 60 + 61, 2 * vd * vd + (nc + 1) * 15 + 15]]))
        xin = x if dtype == torch.float64 else x.astype(np.float32).astype(np.float64)
        ref = sample_Kx(mesh, xin, dofs, gamma=1e3, rho=1.0)
        err = np.linalg.norm(y[dofs] - ref) / np.linalg.norm(ref)
        assert err < tol, L
        cw = _compwise(y[dofs], ref, sample_abs_Kx(mesh, xin, dofs, gamma=1e3, rho=1.0))
        assert cw < (1e-12 if dtype == torch.float64 else 1e-4), (L, cw)
    gpu.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_full_size_2d_512_chebyshev_sampled_rows(dtype, tol):
    """The kernel of the benchmark's roofline entry at full size: the FP32 /
    FP64 Chebyshev application for A (k_A = 1) on the 512^2 level through
    smg_chebyshev, on sampled rows against the oracle's recurrence (with k_A
    = 1 a row needs only its own row of A d_0).  The eigenvalue bound is set
    by the test so that both sides use the same one."""
    from paper_2205_15770_amd import StokesMG
    from oracle.mesh import BoxMesh
    from oracle.rows import velocity_stencil, sample_diag_A
    from oracle.smoother import chebyshev_apply, scaling_constant
    gpu = StokesMG(dim=2, fe_degree=2, n_coarse=(8, 8), n_levels=7, gamma=1e3, rho=1.0)
    L = 6
    beta = 2.75
    gpu.set_eigs(L, beta, 1.5)
    nu, _ = gpu.sizes(L)
    r = si.uniform(nu, 123)
    y = gpu.chebyshev(L, 0, _dev(r, dtype)).cpu().numpy().astype(np.float64)
    mesh = BoxMesh(2, (512, 512), 2)
    rng = np.random.default_rng(8)
    dofs = np.unique(np.concatenate([rng.integers(0, nu, 200), np.arange(0, 20), np.arange(nu - 20, nu),
                                     [1025 * 30 + 30, 1025 * 60 + 61, 1025 * 1025 + 1025 * 7 + 13]]))
    need = velocity_stencil(mesh, dofs)
    dinv = np.ones(nu)
    dinv[need] = 1.0 / sample_diag_A(mesh, need, gamma=1e3, rho=1.0)
    rin = r if dtype == torch.float64 else r.astype(np.float32).astype(np.float64)

    def rows_of_A(v):   # A v on the sampled rows (the only rows the result is read at)
        out = np.zeros(nu)
        out[dofs] = sample_Kx(mesh, np.concatenate([v, np.zeros(mesh.n_pnode)]), dofs, gamma=1e3, rho=1.0)
        return out

    ref = scaling_constant(1) * chebyshev_apply(rows_of_A, dinv, rin, 1, beta)
    assert np.linalg.norm(y[dofs] - ref[dofs]) / np.linalg.norm(ref[dofs]) < tol
    gpu.close()


_CHEB3D_REF = {}


def _cheb3d_64_reference(beta):
    """Sampled rows of sigma Cheb(A, D_A, 1) r on the 64^3 level from the
    oracle (rows, their stencils' diagonal, the recurrence), computed once for
    both kernel variants."""
    if beta in _CHEB3D_REF:
        return _CHEB3D_REF[beta]
    from oracle.mesh import BoxMesh
    from oracle.rows import velocity_stencil, sample_diag_A
    from oracle.smoother import chebyshev_apply, scaling_constant
    mesh = BoxMesh(3, (64, 64, 64), 2)
    vd = 129
    Nv = vd ** 3
    nu = 3 * Nv
    r = si.uniform(nu, 124)
    rng = np.random.default_rng(9)
    pts = [(x_, y_, z) for x_ in (1, 15, 16, 17, 31, 32, 33, 64, 127) for y_ in (1, 11, 12, 13, 15, 16, 17, 127)
           for z in (1, 13, 14, 15, 63, 127)]
    extra = [c * Nv + vd * vd * z + vd * y_ + x_ for c in range(3) for (x_, y_, z) in pts[::7]]
    dofs = np.unique(np.concatenate([rng.integers(0, nu, 100), np.arange(0, 10), np.arange(nu - 10, nu), extra]))
    need = velocity_stencil(mesh, dofs)
    dinv = np.ones(nu)
    dinv[need] = 1.0 / sample_diag_A(mesh, need)
    rin = r.astype(np.float32).astype(np.float64)

    def rows_of_A(v):   # A v on the sampled rows (the only rows the result is read at)
        out = np.zeros(nu)
        out[dofs] = sample_Kx(mesh, np.concatenate([v, np.zeros(mesh.n_pnode)]), dofs)
        return out

    ref = scaling_constant(1) * chebyshev_apply(rows_of_A, dinv, rin, 1, beta)
    _CHEB3D_REF[beta] = (r, dofs, ref[dofs])
    return _CHEB3D_REF[beta]


@pytest.mark.parametrize("variant", ["column_sweep", "matrix_cores"])
def test_full_size_3d_64_chebyshev_sampled_rows(variant):
    """The FP32 Chebyshev application for A (k_A = 1) on the 64^3 level of the
    3D workload at full size through smg_chebyshev -- on the column sweep (the
    default) and on the matrix-core cell kernel -- on sampled rows against the
    oracle's recurrence (with k_A = 1 a row needs only its own row of A d_0).
    The rows include nodes on the tile and z-chunk boundaries of both kernels
    and on the domain faces, in all three components.  The eigenvalue bound
    is set by the test so that both sides use the same one."""
    from paper_2205_15770_amd import StokesMG
    beta = 2.6
    r, dofs, ref = _cheb3d_64_reference(beta)
    env = {"SMG_MFMA3D_MIN_N": "64" if variant == "matrix_cores" else "0"}
    with _env({"env": env}):
        gpu = StokesMG(dim=3, fe_degree=2, n_coarse=(2, 2, 2), n_levels=6, mu=1.0, gamma=0.0)
    L = 5
    gpu.set_eigs(L, beta, 1.5)
    nu, _ = gpu.sizes(L)
    assert nu == len(r)
    y = gpu.chebyshev(L, 0, _dev(r, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(y[dofs] - ref) / np.linalg.norm(ref) < 2e-5
    gpu.close()


def _sampled_dofs(n, nu, lat_v, extra, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, n, 400), np.arange(0, 40), np.arange(n - 40, n),
                                     np.arange(nu - 20, nu + 20), extra]))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_full_size_3d_64_sampled_rows(dtype, tol):
    """The 64^3 Q2-Q1 workload (6 levels) at full size: sampled rows of K x on
    the finest level (column-sweep kernel) and on the 32^3 level (cell-block
    kernel) against the oracle's row-by-row definition."""
    from paper_2205_15770_amd import StokesMG
    from oracle.mesh import BoxMesh
    gpu = StokesMG(dim=3, fe_degree=2, n_coarse=(2, 2, 2), n_levels=6, mu=1.0, gamma=0.0)
    for L, nc in ((5, 64), (4, 32)):
        n = gpu.n_total(L)
        nu, _ = gpu.sizes(L)
        x = si.uniform(n, 98 + L)
        y = gpu.vmult(L, _dev(x, dtype)).cpu().numpy().astype(np.float64)
        mesh = BoxMesh(3, (nc, nc, nc), 2)
        vd = 2 * nc + 1
        # nodes on tile and chunk boundaries of both kernels, and on the faces
        extra = [vd * vd * z + vd * y_ + x_ for (x_, y_, z) in
                 [(14, 14, 14), (15, 7, 30), (6, 6, 6), (7, 13, 2 * nc - 1), (1, 1, 1), (vd - 2, vd - 2, vd - 2)]]
        dofs = _sampled_dofs(n, nu, vd, extra + [nu // 3 + e for e in extra], 6 + L)
        xin = x if dtype == torch.float64 else x.astype(np.float32).astype(np.float64)
        ref = sample_Kx(mesh, xin, dofs)
        assert np.linalg.norm(y[dofs] - ref) / np.linalg.norm(ref) < tol, L
        cw = _compwise(y[dofs], ref, sample_abs_Kx(mesh, xin, dofs))
        assert cw < (1e-12 if dtype == torch.float64 else 1e-4), (L, cw)
    gpu.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_full_size_3d_q3_32_perturbed_sampled_rows(dtype, tol):
    """The 32^3 Q3-Q2 workload with perturbed vertices (seed 4) and Fourier
    viscosity in [1, 100] (seed 5), 5 levels, at full size: sampled rows of
    K x on the finest level (quadrature-point kernel)."""
    from paper_2205_15770_amd import StokesMG
    from oracle.mesh import BoxMesh
    V = si.perturbed_box_vertices(32, dim=3, amplitude=0.2, seed=4)
    mu = si.fourier_log_viscosity(32, dim=3, seed=5)
    gpu = StokesMG(dim=3, fe_degree=3, n_coarse=(2, 2, 2), n_levels=5, mu_cell=mu, gamma=0.0, fine_vertices=V)
    L = 4
    n = gpu.n_total(L)
    nu, _ = gpu.sizes(L)
    x = si.uniform(n, 97)
    y = gpu.vmult(L, _dev(x, dtype)).cpu().numpy().astype(np.float64)
    mesh = BoxMesh(3, (32, 32, 32), 3, vertices=V, mu_cell=mu)
    vd = 97
    extra = [vd * vd * z + vd * y_ + x_ for (x_, y_, z) in [(3, 3, 3), (4, 50, 61), (95, 95, 95), (48, 1, 2)]]
    dofs = _sampled_dofs(n, nu, vd, extra, 16)
    xin = x if dtype == torch.float64 else x.astype(np.float32).astype(np.float64)
    ref = sample_Kx(mesh, xin, dofs)
    assert np.linalg.norm(y[dofs] - ref) / np.linalg.norm(ref) < tol
    cw = _compwise(y[dofs], ref, sample_abs_Kx(mesh, xin, dofs))
    assert cw < (1e-12 if dtype == torch.float64 else 1e-4), cw
    gpu.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_graph_replayed_cycle_matches_eager(precision):
    """The preconditioning cycle inside smg_solve is captured into a HIP graph
    and replayed; with kernel timing on it runs eagerly.  Replays (with eager
    work and synchronisation in between) must equal the eager result."""
    from paper_2205_15770_amd import StokesMG
    cfg = CONFIGS["2d_k2"]
    gpu = StokesMG(dim=2, fe_degree=2, n_coarse=cfg["n_coarse"], n_levels=cfg["levels"], gamma=3.0,
                   precision=precision)
    L = cfg["levels"] - 1
    n = gpu.n_total(L)
    ora, _ = _setup("2d_k2")
    b = _dev(ora.levels[L].rhs_from_nodal_f(si.nodal_random_f(2, ora.meshes[L].n_vnode, seed=4)))
    gpu.profile(True)                       # eager launches
    x_e = torch.zeros(n, dtype=torch.float64, device="cuda")
    info_e = gpu.solve(x_e, b, rtol=1e-9, maxit=60)
    gpu.profile(False)                      # graph replay
    for rep in range(3):
        x_g = torch.zeros(n, dtype=torch.float64, device="cuda")
        info_g = gpu.solve(x_g, b, rtol=1e-9, maxit=60)
        torch.cuda.synchronize()
        y = gpu.vmult(L, x_g)               # eager work between replays
        torch.cuda.synchronize()
        assert info_g["iterations"] == info_e["iterations"]
        assert torch.equal(x_g, x_e), rep
    gpu.close()


@pytest.mark.parametrize("case", ["2d_512", "3d_32"])
def test_full_size_cycle_against_oracle(case):
    """One whole V-cycle on a full benchmark hierarchy against the oracle's
    cycle (Algorithm 1 with the inexact symmetric Uzawa smoother, the
    oracle's Lanczos bounds injected): the 512^2 Q2-Q1 workload (7 levels,
    gamma = 1e3, 2,364,419 DoFs) and the 3D Q2-Q1 hierarchy on 32^3 (5
    levels, gamma = 0, 859,812 DoFs; 64^3 does not fit the oracle's
    assembled matrices), from a non-zero start, FP64 and FP32 cycles, with the
    kernel choices the solvers make at these sizes (two-stage fused launches
    on every 2D level, three-stage up to 128^2; column sweep and cell blocks
    in 3D)."""
    from paper_2205_15770_amd import StokesMG
    from oracle.mesh import make_hierarchy
    from oracle.mg import Multigrid
    dim, nc, lv, g = (2, (8, 8), 7, 1e3) if case == "2d_512" else (3, (2, 2, 2), 5, 0.0)
    ora = Multigrid(make_hierarchy(dim, nc, lv, 2), mu=1.0, gamma=g, rho=1.0, k_A=1, k_S=1, smooth_steps=2,
                    cycle_index=1)
    L = ora.L
    n = ora.levels[L].K.shape[0]
    b = ora.levels[L].rhs_from_nodal_f(si.nodal_random_f(dim, ora.meshes[L].n_vnode, seed=5))
    x0 = si.uniform(n, 75) * 0.1
    x0[ora.levels[L].constrained] = 0.0
    ref = ora.cycle(L, x0.copy(), b)
    for prec, dt, tol in (("f64", torch.float64, 1e-10), ("f32", torch.float32, 1e-4)):
        gpu = StokesMG(dim=dim, fe_degree=2, n_coarse=nc, n_levels=lv, mu=1.0, rho=1.0, gamma=g, cheb_deg_A=1,
                       cheb_deg_S=1, smooth_steps=2, cycle_index=1, schur_diag="d", precision=prec)
        _inject_betas(ora, gpu)
        xg = _dev(x0, dt)
        gpu.vcycle(L, xg, _dev(b, dt))
        torch.cuda.synchronize()
        err = _rel(xg, ref)
        assert err < tol, (prec, err)
        gpu.close()
