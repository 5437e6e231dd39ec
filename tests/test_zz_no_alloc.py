"""smg_vmult_noalloc (the allocation-free variant of smg_vmult) through the C
ABI against smg_vmult on the same context: vertex-given cells, whose kernels
keep per-cell partial results in the fixed device buffer, and box cells,
which need none.  Two calls in a row, the second on a smaller level, so the
shared buffer holds the first call's results when the second one starts.
Bar: FP64 relative 2-norm difference <= 1e-12, FP32 <= 2e-5 (the same
kernels run, so the results are expected to be identical)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth_inputs as si

pytestmark = pytest.mark.gpu

CASES = {
    "3d_k3_pert": dict(dim=3, k=3, n_coarse=(2, 2, 2), levels=3, pert=True),
    "2d_k2_pert": dict(dim=2, k=2, n_coarse=(3, 2), levels=4, pert=True),
    "3d_k2_box": dict(dim=3, k=2, n_coarse=(2, 3, 2), levels=3, pert=False),
}


def _solver(cfg, **kw):
    from paper_2205_15770_amd import StokesMG
    n_f = [c * 2 ** (cfg["levels"] - 1) for c in cfg["n_coarse"]]
    V = si.perturbed_box_vertices(n_f, dim=cfg["dim"], amplitude=0.2, seed=21) if cfg["pert"] else None
    mu = si.uniform(int(np.prod(n_f)), 17, 0.5, 3.0)
    return StokesMG(dim=cfg["dim"], fe_degree=cfg["k"], n_coarse=cfg["n_coarse"], n_levels=cfg["levels"],
                    mu_cell=mu, gamma=7.0, rho=0.5, fine_vertices=V, **kw)


def _noalloc(mg, level, x, y):
    from paper_2205_15770_amd import _lib
    code = 0 if x.dtype == torch.float64 else 1
    return mg.lib.smg_vmult_noalloc(mg._h, level, code, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()))


def _rel(a, b):
    return (torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double())).item()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_vmult_noalloc_matches_vmult(name, dtype, tol):
    from paper_2205_15770_amd import _lib
    cfg = CASES[name]
    mg = _solver(cfg)
    L = cfg["levels"] - 1
    for level, seed in ((L, 5), (L - 1, 6)):     # the second call on a smaller level
        n = mg.n_total(level)
        print(f"case {name} {dtype} level {level} n {n}", flush=True)
        x = torch.tensor(si.uniform(n, seed), dtype=dtype, device="cuda")
        y_ref = mg.vmult(level, x)
        y = torch.full((n,), float("nan"), dtype=dtype, device="cuda")
        assert _noalloc(mg, level, x, y) == _lib.SMG_OK, _lib.last_error()
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert _rel(y, y_ref) <= tol, (name, level)
    mg.close()


def test_vmult_noalloc_rejects_levels_beyond_the_buffer():
    """320^2 vertex-given Q2 cells need 17.3 MiB of partial results in FP64:
    rejected before any device work; the 160^2 level below fits."""
    from paper_2205_15770_amd import _lib
    cfg = dict(dim=2, k=2, n_coarse=(5, 5), levels=7, pert=True)
    mg = _solver(cfg)
    L = cfg["levels"] - 1
    n = mg.n_total(L)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert _noalloc(mg, L, x, y) == _lib.SMG_EINVAL
    assert "bytes of scratch" in _lib.last_error()
    n = mg.n_total(L - 1)
    x = torch.tensor(si.uniform(n, 8), dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert _noalloc(mg, L - 1, x, y) == _lib.SMG_OK, _lib.last_error()
    assert _rel(y, mg.vmult(L - 1, x)) <= 1e-12
    mg.close()
