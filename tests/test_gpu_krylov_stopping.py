"""Stopping rules of the FP64 FGMRES outer solve (host loop).

A solve stopped by its iteration limit, or by a tolerance that falls between
two iterates, must retrace the unconstrained run: the same iterations and the
same residual history up to the stopping point, whatever the host had queued
for an iteration that then does not run.  The last entry of a stopped run is
the recomputed true residual, the unconstrained run's entry at that index the
FGMRES estimate, so that entry is compared loosely.  Restart lengths 30 and 3
(the latter stops inside and at the end of restart cycles).
"""
import numpy as np
import pytest
import torch

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _problem(precision, restart):
    from paper_2205_15770_amd import StokesMG, SMG_BLOCK_MASS
    mg = StokesMG(dim=2, fe_degree=2, n_coarse=(5, 3), n_levels=4, gamma=7.0, rho=0.5, c_pressure=0.2,
                  precision=precision, fgmres_restart=restart)
    L = mg.n_levels - 1
    nu, npr = mg.sizes(L)
    f = torch.tensor(si.nodal_random_f(2, nu // 2, seed=4).ravel(), dtype=torch.float64, device="cuda")
    b = torch.zeros(nu + npr, dtype=torch.float64, device="cuda")
    mg.apply_block(L, SMG_BLOCK_MASS, f, b[:nu])
    return mg, b


def _run(mg, b, rtol, maxit):
    x = torch.zeros_like(b)
    info = mg.solve(x, b, rtol=rtol, maxit=maxit, raise_on_failure=False)
    return info, x


@pytest.mark.parametrize("restart", [30, 3])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_fgmres_stopping_rules(precision, restart):
    mg, b = _problem(precision, restart)
    full, _ = _run(mg, b, 1e-13, 60)
    H = full["history"]
    n = full["iterations"]
    assert n >= 5 and len(H) == n + 1
    assert np.all(np.diff(H[:4]) < 0)

    def same_prefix(h):
        k = len(h) - 1
        assert np.allclose(h[:k], H[:k], rtol=1e-12, atol=0.0)
        assert abs(h[k] - H[k]) <= 1e-3 * H[k]

    # iteration limit
    for k in range(1, 6):
        info, _ = _run(mg, b, 1e-13, k)
        assert info["iterations"] == k, k
        assert len(info["history"]) == k + 1
        same_prefix(info["history"])
    # tolerance between two iterates (three times above the later one)
    for k in range(0, 4):
        rtol = 3.0 * H[k + 1]
        assert rtol < H[k]
        info, x = _run(mg, b, rtol, 60)
        assert info["status"] == 0
        assert info["iterations"] == k + 1, (k, info["iterations"])
        same_prefix(info["history"])
        assert info["rel_residual"] <= rtol
        # the true residual of the returned iterate
        L = mg.n_levels - 1
        r = mg.residual(L, x, b)
        assert torch.linalg.norm(r).item() <= 1.0001 * rtol * torch.linalg.norm(b).item()
    mg.close()
