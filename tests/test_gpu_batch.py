"""Batched solves (smg_batch_*): the stages of the multigrid cycle and of the
Krylov iteration run for all problems of a batch in packed launches (one
graph launch per batched cycle).  Each problem must come out exactly as
solved alone (the same kernels in the same order on its data, the same
reductions), and small problems are checked against the oracle: their
operator, the batched cycle and the batched solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _problems(prec):
    # uneven sizes (side counts c 2^(levels-1) from 8 to 112) and gamma from 0 to 1e4
    return [dict(dim=2, fe_degree=2, n_coarse=(c, c), n_levels=lv, gamma=g, rho=1.0, precision=prec)
            for (c, lv, g) in [(4, 3, 0.0), (5, 2, 1e4), (6, 3, 37.0), (7, 5, 5e3), (4, 4, 2e3), (3, 3, 10.0),
                               (2, 3, 1.0)]]


def _rhs(mg, seed):
    from paper_2205_15770_amd import SMG_BLOCK_MASS
    L = mg.n_levels - 1
    nu, np_ = mg.sizes(L)
    f = torch.tensor(si.nodal_random_f(2, nu // 2, seed=seed).ravel(), dtype=torch.float64, device="cuda")
    b = torch.zeros(nu + np_, dtype=torch.float64, device="cuda")
    mg.apply_block(L, SMG_BLOCK_MASS, f, b[:nu])
    torch.cuda.synchronize()
    return b


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("wgf", [False, True])
def test_batch_solve_equals_individual_solves(prec, wgf, monkeypatch):
    """wgf: the fused launches of every level on workgroups of 2 x 2 waves
    (by default only levels of 512 cells per direction), packed through
    their own launch functor in the batch."""
    from paper_2205_15770_amd import StokesMG, StokesBatch
    if wgf:
        monkeypatch.setenv("SMG_WGF2D_MIN_N", "1")
    probs = _problems(prec)
    batch = StokesBatch(probs)
    nl, var = batch.info()
    assert nl > 0 and var == 0
    bs = [_rhs(mg, 80 + i) for i, mg in enumerate(batch.solvers)]
    xs = [torch.zeros_like(b) for b in bs]
    infos = batch.solve(xs, bs, rtol=1e-9, maxit=200)
    for i, p in enumerate(probs):
        mg = StokesMG(**p)
        x1 = torch.zeros_like(bs[i])
        info = mg.solve(x1, bs[i], rtol=1e-9, maxit=200)
        assert infos[i]["iterations"] == info["iterations"], i
        assert infos[i]["rel_residual"] <= 1e-9
        assert np.array_equal(infos[i]["history"], info["history"]), i
        assert torch.equal(xs[i], x1), i
        mg.close()
    # a second solve on the same batch (plans and graph re-used) from a non-zero guess
    x0 = [x.clone() * 0.5 for x in xs]
    infos2 = batch.solve(x0, bs, rtol=1e-9, maxit=200)
    assert all(inf["rel_residual"] <= 1e-9 for inf in infos2)
    batch.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_precondition_equals_individual_cycles(prec):
    from paper_2205_15770_amd import StokesBatch
    batch = StokesBatch(_problems(prec))
    vs = [torch.tensor(si.uniform(m.n_total(m.n_levels - 1), 300 + i), dtype=torch.float64, device="cuda")
          for i, m in enumerate(batch.solvers)]
    zs = batch.precondition(vs)
    for i, m in enumerate(batch.solvers):
        L = m.n_levels - 1
        dt = torch.float32 if prec == "f32" else torch.float64
        x = torch.zeros(m.n_total(L), dtype=dt, device="cuda")
        m.vcycle(L, x, vs[i].to(dt))
        torch.cuda.synchronize()
        assert torch.equal(zs[i], x.to(torch.float64)), i
    batch.close()


def test_batch_small_problems_against_oracle():
    """Small problems (per-cell viscosity, C = 0, uneven sizes and gamma):
    each problem's operator, its cycle inside the batched cycle (FP64, with
    the oracle's eigenvalue bounds) and its batched solve against the oracle
    (direct solve of the bordered system)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from paper_2205_15770_amd import StokesMG, StokesBatch
    from oracle.mesh import make_hierarchy
    from oracle.mg import Multigrid
    specs = [((3, 2), 2, 7.0), ((2, 3), 3, 0.0), ((4, 4), 2, 1e3)]
    oras, mgs = [], []
    for k, (nc, lv, g) in enumerate(specs):
        n_f = [c * 2 ** (lv - 1) for c in nc]
        mu = si.uniform(int(np.prod(n_f)), 17 + k, 0.5, 3.0)
        ora = Multigrid(make_hierarchy(2, nc, lv, 2, fine_mu=mu), mu=1.0, gamma=g, rho=0.5, k_A=1, k_S=1,
                        smooth_steps=2, cycle_index=1)
        mg = StokesMG(dim=2, fe_degree=2, n_coarse=nc, n_levels=lv, mu_cell=mu, gamma=g, rho=0.5, precision="f64")
        for l in range(1, lv):
            mg.set_eigs(l, ora.smoothers[l].beta_A, ora.smoothers[l].beta_S)
        oras.append(ora)
        mgs.append(mg)
    batch = StokesBatch.from_solvers(mgs)
    vs, bs = [], []
    for k, (ora, mg) in enumerate(zip(oras, mgs)):
        L = ora.L
        K = ora.levels[L].K
        x = si.uniform(K.shape[0], 400 + k)
        y = mg.vmult(L, torch.tensor(x, dtype=torch.float64, device="cuda")).cpu().numpy()
        assert np.linalg.norm(y - K @ x) <= 1e-12 * np.linalg.norm(K @ x)
        b = ora.levels[L].rhs_from_nodal_f(si.nodal_random_f(2, ora.meshes[L].n_vnode, seed=500 + k))
        vs.append(torch.tensor(b, dtype=torch.float64, device="cuda"))
        bs.append(b)
    zs = batch.precondition(vs)
    for k, ora in enumerate(oras):
        zo = ora.cycle(ora.L, np.zeros(len(bs[k])), bs[k])
        assert np.linalg.norm(zs[k].cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo), k
    xs = [torch.zeros_like(v) for v in vs]
    infos = batch.solve(xs, vs, rtol=1e-10, maxit=100)
    for k, ora in enumerate(oras):
        asm = ora.levels[ora.L]
        nu = asm.A.shape[0]
        n = asm.K.shape[0]
        m = np.zeros(n)
        m[nu:] = asm.Mp @ np.ones(n - nu)
        Kb = sp.bmat([[asm.K, sp.csr_matrix(m[:, None])], [sp.csr_matrix(m[None, :]), None]]).tocsc()
        xd = spla.spsolve(Kb, np.concatenate([bs[k], [0.0]]))[:-1]
        xg = xs[k].cpu().numpy()
        assert infos[k]["rel_residual"] <= 1e-10
        assert np.linalg.norm(bs[k] - asm.K @ xg) <= 1.05e-10 * np.linalg.norm(bs[k])
        assert np.linalg.norm(xg - xd) <= 1e-6 * np.linalg.norm(xd), k
    batch.close()


def test_batch_autotune_keeps_solutions():
    from paper_2205_15770_amd import StokesBatch
    batch = StokesBatch(_problems("f32"))
    bs = [_rhs(mg, 90 + i) for i, mg in enumerate(batch.solvers)]
    x_ref = [torch.zeros_like(b) for b in bs]
    ref = batch.solve(x_ref, bs, rtol=1e-9, maxit=200)
    best, times = batch.autotune(probe_cycles=3)
    assert 0 <= best < len(times) and all(t > 0 for t in times)
    assert batch.info()[1] == best
    xs = [torch.zeros_like(b) for b in bs]
    infos = batch.solve(xs, bs, rtol=1e-9, maxit=200)
    for i in range(len(bs)):
        assert infos[i]["rel_residual"] <= 1e-9
        assert abs(infos[i]["iterations"] - ref[i]["iterations"]) <= 1
        rel = (torch.linalg.norm(xs[i] - x_ref[i]) / torch.linalg.norm(x_ref[i])).item()
        assert rel <= 1e-6, (i, rel)
    batch.close()


def test_batch_rejects_what_it_does_not_pack():
    from paper_2205_15770_amd import StokesMG, StokesBatch, SmgError
    a = StokesMG(dim=2, fe_degree=2, n_coarse=(3, 3), n_levels=2, precision="f32")
    b = StokesMG(dim=2, fe_degree=2, n_coarse=(4, 4), n_levels=2, precision="f64")
    c = StokesMG(dim=3, fe_degree=2, n_coarse=(2, 2, 2), n_levels=2)
    with pytest.raises(SmgError):
        StokesBatch.from_solvers([a, b])      # two preconditioner precisions
    with pytest.raises(SmgError):
        StokesBatch.from_solvers([a, c])      # a 3D problem
    with pytest.raises(SmgError):
        StokesBatch.from_solvers([a, a])      # one context twice
    for m in (a, b, c):
        m.close()
