"""Non-homogeneous Dirichlet data on the GPU (smg_lift_dirichlet,
smg_insert_dirichlet) against the oracle's lifting, a solution in the
discrete spaces reproduced from its boundary values, and the driven cavity
against the oracle's direct solve.

Tolerances: the lift is one operator application (FP64 <= 1e-12 relative,
FP32 <= 2e-5); the insertion is a copy (exact); solves to rtol 1e-12 carry
errors of order cond(K) * 1e-12, so solutions agree to <= 1e-8."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth_inputs as si
from oracle.mesh import BoxMesh, make_hierarchy
from oracle.assemble import Assembled
from oracle.adjoint import bordered_solve
from oracle.dirichlet import lift, insert, lid_driven_cavity

pytestmark = pytest.mark.gpu

CASES = {
    "2d_k2": dict(dim=2, k=2, n_coarse=(5, 3), levels=3),
    "2d_k3": dict(dim=2, k=3, n_coarse=(3, 2), levels=3),
    "3d_k2": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3),
    "2d_k2_plain": dict(dim=2, k=2, n_coarse=(5, 3), levels=3, env={"SMG_SPLIT2D_MAX_N": "0", "SMG_FUSE2D_MAX_N": "0"}),
    "3d_k2_sweep": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3, env={"SMG_BLOCK3D_MAX_N": "0"}),
    "3d_k2_cellblock": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3, env={"SMG_PLANE3D_MAX_N": "0"}),
    "3d_k3": dict(dim=3, k=3, n_coarse=(2, 2, 3), levels=2),
    "2d_k2_pert": dict(dim=2, k=2, n_coarse=(3, 2), levels=3, pert=True),
    "3d_k3_pert": dict(dim=3, k=3, n_coarse=(2, 2, 2), levels=2, pert=True),
}
GAMMA, RHO, CP = 4.0, 0.5, 0.3


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    a = a.detach().cpu().numpy().astype(np.float64) if torch.is_tensor(a) else a
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _pair(name, monkeypatch):
    from paper_2205_15770_amd import StokesMG
    c = CASES[name]
    dim, k, L = c["dim"], c["k"], c["levels"]
    n_f = [v * 2 ** (L - 1) for v in c["n_coarse"]]
    mu_cell = si.uniform(int(np.prod(n_f)), 23, 0.5, 3.0)
    V = si.perturbed_box_vertices(n_f, dim=dim, amplitude=0.2, seed=29) if c.get("pert") else None
    for k_, v_ in c.get("env", {}).items():
        monkeypatch.setenv(k_, v_)
    gpu = StokesMG(dim=dim, fe_degree=k, n_coarse=c["n_coarse"], n_levels=L, mu_cell=mu_cell, gamma=GAMMA,
                   rho=RHO, c_pressure=CP, fine_vertices=V)
    mesh = make_hierarchy(dim, c["n_coarse"], L, k, fine_mu=mu_cell, fine_vertices=V)[-1]
    asm = Assembled(mesh, gamma=GAMMA, rho=RHO, c_p=CP)
    return gpu, asm, L - 1


@pytest.mark.parametrize("name", list(CASES))
def test_lift_and_insert_match_oracle(name, monkeypatch):
    gpu, asm, L = _pair(name, monkeypatch)
    nu, n = asm.A.shape[0], asm.K.shape[0]
    ud = si.uniform(nu, 31)
    b = si.uniform(n, 32)
    ref = lift(asm, b, ud)
    bg = _dev(b)
    gpu.lift_dirichlet(L, _dev(ud), bg)
    assert _rel(bg, ref) < 1e-12
    b32 = _dev(b, torch.float32)
    gpu.lift_dirichlet(L, _dev(ud, torch.float32), b32)
    ref32 = lift(asm, b.astype(np.float32).astype(np.float64), ud.astype(np.float32).astype(np.float64))
    assert _rel(b32, ref32) < 2e-5
    x0 = si.uniform(n, 33)
    xg = _dev(x0)
    gpu.insert_dirichlet(L, _dev(ud), xg)
    assert np.array_equal(xg.cpu().numpy(), insert(asm, x0, ud))
    gpu.close()


@pytest.mark.parametrize("dim,k,n_coarse,levels", [(2, 2, (3, 2), 4), (2, 3, (2, 2), 3), (3, 2, (2, 2, 2), 3)])
def test_solution_in_discrete_space_from_boundary_values(dim, k, n_coarse, levels):
    """u quadratic with div u = 0 and non-zero boundary values, p linear with
    zero mean, constant mu, f = -mu Lap u + gamma rho u + grad p (quadratic, so
    its nodal interpolant is exact and M_v f is the exact load vector): the
    lifted solve must return u and p at the nodes."""
    from paper_2205_15770_amd import StokesMG, SMG_BLOCK_MASS
    mu, gr = 1.3, 2.0
    gpu = StokesMG(dim=dim, fe_degree=k, n_coarse=n_coarse, n_levels=levels, mu=mu, gamma=gr, rho=1.0)
    L = levels - 1
    mesh = BoxMesh(dim, [v * 2 ** L for v in n_coarse], k)
    X = mesh.velocity_node_coordinates()
    if dim == 2:
        U = np.stack([X[:, 1] ** 2, X[:, 0] ** 2], axis=1)
    else:
        U = np.stack([X[:, 1] ** 2 + X[:, 2] ** 2, X[:, 0] ** 2 + X[:, 2] ** 2, X[:, 0] ** 2 + X[:, 1] ** 2], axis=1)
    F = -mu * 2.0 * (dim - 1) + gr * U + 1.0
    u_nodal = U.T.ravel()
    pidx = mesh._unflat(np.arange(mesh.n_pnode), mesh.p_dims)
    p_nodal = (pidx / np.array([(k - 1) * v for v in mesh.n], dtype=np.float64)).sum(axis=1) - 0.5 * dim
    nu, np_ = gpu.sizes(L)
    b = torch.zeros(nu + np_, dtype=torch.float64, device="cuda")
    gpu.apply_block(L, SMG_BLOCK_MASS, _dev(F.T.ravel()), b[:nu])
    ud = _dev(u_nodal)
    gpu.lift_dirichlet(L, ud, b)
    x = torch.zeros_like(b)
    gpu.solve(x, b, rtol=1e-12, maxit=100)
    gpu.insert_dirichlet(L, ud, x)
    xs = x.cpu().numpy()
    assert np.max(np.abs(xs[:nu] - u_nodal)) < 1e-8 * np.max(np.abs(u_nodal))
    assert np.max(np.abs(xs[nu:] - p_nodal)) < 1e-8 * np.max(np.abs(p_nodal)) * 10
    gpu.close()


@pytest.mark.parametrize("dim,n_coarse,levels", [(2, (4, 4), 3), (3, (2, 2, 2), 3)])
def test_driven_cavity_matches_oracle_direct_solve(dim, n_coarse, levels):
    from paper_2205_15770_amd import StokesMG
    gpu = StokesMG(dim=dim, fe_degree=2, n_coarse=n_coarse, n_levels=levels, mu=1.0)
    L = levels - 1
    mesh = BoxMesh(dim, [v * 2 ** L for v in n_coarse], 2)
    asm = Assembled(mesh)
    ud = lid_driven_cavity(mesh)
    ref = insert(asm, bordered_solve(asm, lift(asm, np.zeros(asm.K.shape[0]), ud)), ud)
    udg = _dev(ud)
    b = torch.zeros(asm.K.shape[0], dtype=torch.float64, device="cuda")
    gpu.lift_dirichlet(L, udg, b)
    x = torch.zeros_like(b)
    info = gpu.solve(x, b, rtol=1e-12, maxit=100)
    gpu.insert_dirichlet(L, udg, x)
    assert info["iterations"] < 40
    assert _rel(x, ref) < 1e-8
    gpu.close()
