"""Batched solves (smg_batch_solve, smg_batch_autotune): every instance of a
batch solved concurrently by several host threads on its own stream must give
exactly the result of solving it alone (the kernels are deterministic)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _problems():
    return [dict(dim=2, fe_degree=2, n_coarse=(c, c), n_levels=lv, gamma=g, rho=1.0, precision=p)
            for (c, lv, g, p) in [(4, 3, 0.0, "f32"), (5, 2, 1e4, "f64"), (6, 3, 37.0, "f32"), (7, 2, 5e3, "f32"),
                                  (4, 4, 2e3, "f64")]]


def _rhs(mg, seed):
    from paper_2205_15770_amd import SMG_BLOCK_MASS
    L = mg.n_levels - 1
    nu, np_ = mg.sizes(L)
    f = torch.tensor(si.nodal_random_f(2, nu // 2, seed=seed).ravel(), dtype=torch.float64, device="cuda")
    b = torch.zeros(nu + np_, dtype=torch.float64, device="cuda")
    mg.apply_block(L, SMG_BLOCK_MASS, f, b[:nu])
    torch.cuda.synchronize()
    return b


def test_batch_equals_individual_solves():
    from paper_2205_15770_amd import StokesMG, StokesBatch
    probs = _problems()
    batch = StokesBatch(probs)
    bs = [_rhs(mg, 80 + i) for i, mg in enumerate(batch.solvers)]
    xs = [torch.zeros_like(b) for b in bs]
    best, times = batch.autotune(xs, bs, candidates=(1, 2, 3))
    assert best in (1, 2, 3) and len(times) == 3
    for x in xs:
        x.zero_()
    infos = batch.solve(xs, bs, rtol=1e-9, maxit=200, nthreads=3)
    for i, p in enumerate(probs):
        mg = StokesMG(**p)
        x1 = torch.zeros_like(bs[i])
        info = mg.solve(x1, bs[i], rtol=1e-9, maxit=200)
        assert infos[i]["iterations"] == info["iterations"]
        assert infos[i]["rel_residual"] <= 1e-9
        assert torch.equal(xs[i], x1), i
        mg.close()
    batch.close()


def test_batch_rejects_repeated_context():
    from paper_2205_15770_amd import StokesBatch, SmgError
    batch = StokesBatch(_problems()[:2])
    bs = [_rhs(mg, 90 + i) for i, mg in enumerate(batch.solvers)]
    xs = [torch.zeros_like(b) for b in bs]
    batch.solvers = [batch.solvers[0], batch.solvers[0]]
    with pytest.raises(SmgError):
        batch.solve([xs[0], xs[0]], [bs[0], bs[0]])
    batch.close()
