"""Matrix-free monolithic geometric multigrid for Q_k-Q_{k-1} Taylor-Hood
Stokes and generalized Stokes problems on MI355X (gfx950).

Thin Python binding over the C ABI of ``libsmg.so`` (``include/smg.h``):
argument marshalling only.  Vectors are torch tensors on the GPU (float64 or
float32) in the layout [u_1 | ... | u_d | p] of each level; torch supplies
device memory and the stream, every computation runs in the library's HIP
kernels.  If the library is not built, constructing a solver raises.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (SMG_F64, SMG_F32, SMG_BLOCK_K, SMG_BLOCK_A, SMG_BLOCK_BT, SMG_BLOCK_B,
                   SMG_BLOCK_MASS, SMG_BLOCK_MP, SMG_SCHUR_D, SMG_SCHUR_LOC, SMG_SCHUR_P, SMG_SCHUR_EXACT, SmgError)

__all__ = ["StokesMG", "StokesBatch", "SmgError", "SMG_BLOCK_K", "SMG_BLOCK_A", "SMG_BLOCK_BT", "SMG_BLOCK_B",
           "SMG_BLOCK_MASS", "SMG_BLOCK_MP"]

_SCHUR = {"d": SMG_SCHUR_D, "loc": SMG_SCHUR_LOC, "p": SMG_SCHUR_P, "exact": SMG_SCHUR_EXACT}


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return SMG_F64
    if t.dtype == torch.float32:
        return SMG_F32
    raise TypeError(f"vectors must be float64 or float32, got {t.dtype}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class StokesMG:
    """One multigrid hierarchy (``smg_create``) and its operations."""

    def __init__(self, dim=2, fe_degree=2, n_coarse=(4, 4, 4), n_levels=3, box_lo=(0.0, 0.0, 0.0),
                 box_hi=(1.0, 1.0, 1.0), mu=1.0, mu_cell=None, gamma=0.0, rho=1.0, c_pressure=0.0,
                 cheb_deg_A=1, cheb_deg_S=1, smooth_steps=2, cycle_index=1, schur_diag="d",
                 precision="f64", fgmres_restart=30, stream=None, fine_vertices=None, form="grad"):
        import torch
        self.lib = _lib.load()
        d = _lib.SmgDesc()
        self.lib.smg_desc_default(ctypes.byref(d))
        d.dim, d.fe_degree, d.n_levels = dim, fe_degree, n_levels
        nc = list(n_coarse) + [n_coarse[-1]] * 3
        for a in range(3):
            d.n_coarse[a] = int(nc[a])
            d.box_lo[a] = float((list(box_lo) + [0.0] * 3)[a])
            d.box_hi[a] = float((list(box_hi) + [1.0] * 3)[a])
        d.mu, d.gamma, d.rho, d.c_pressure = float(mu), float(gamma), float(rho), float(c_pressure)
        self._mu_cell = None
        self._verts = None
        if fine_vertices is not None:
            # (n_f + 1)^d vertices x d coordinates, x fastest (read during create)
            self._verts = np.ascontiguousarray(fine_vertices, dtype=np.float64).reshape(-1)
            d.fine_vertices = self._verts.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if mu_cell is not None:
            self._mu_cell = np.ascontiguousarray(mu_cell, dtype=np.float64)
            d.mu_cell = self._mu_cell.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.cheb_deg_A, d.cheb_deg_S = int(cheb_deg_A), int(cheb_deg_S)
        d.smooth_steps, d.cycle_index = int(smooth_steps), int(cycle_index)
        d.schur_diag = _SCHUR[schur_diag] if isinstance(schur_diag, str) else int(schur_diag)
        d.precision = {"f64": 0, "f32": 1}[precision] if isinstance(precision, str) else int(precision)
        d.fgmres_restart = int(fgmres_restart)
        d.form = {"grad": _lib.SMG_FORM_GRAD, "eps": _lib.SMG_FORM_EPS}[form] if isinstance(form, str) else int(form)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        d.stream = ctypes.c_void_p(stream)
        self.desc = d
        self.dim = dim
        self.n_levels = n_levels
        h = ctypes.c_void_p()
        _lib.check(self.lib.smg_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._mu_cell = None
        self._verts = None

    # -- housekeeping ---------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.smg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self, level):
        nu, np_ = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self.lib.smg_sizes(self._h, level, ctypes.byref(nu), ctypes.byref(np_)))
        return nu.value, np_.value

    def n_total(self, level):
        nu, np_ = self.sizes(level)
        return nu + np_

    def _check(self, t, n, name):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous GPU tensor")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, expected {n}")

    def _like(self, ref, n):
        import torch
        return torch.empty(n, dtype=ref.dtype, device=ref.device)

    # -- operators -------------------------------------------------------
    def vmult(self, level, x, y=None):
        n = self.n_total(level)
        self._check(x, n, "x")
        y = self._like(x, n) if y is None else y
        self._check(y, n, "y")
        _lib.check(self.lib.smg_vmult(self._h, level, _dtype_code(x), _ptr(x), _ptr(y)))
        return y

    def residual(self, level, x, b, r=None):
        n = self.n_total(level)
        self._check(x, n, "x")
        self._check(b, n, "b")
        r = self._like(x, n) if r is None else r
        _lib.check(self.lib.smg_residual(self._h, level, _dtype_code(x), _ptr(x), _ptr(b), _ptr(r)))
        return r

    def apply_block(self, level, block, x, y=None):
        nu, np_ = self.sizes(level)
        n_in = {SMG_BLOCK_K: nu + np_, SMG_BLOCK_A: nu, SMG_BLOCK_BT: np_, SMG_BLOCK_B: nu, SMG_BLOCK_MASS: nu,
                SMG_BLOCK_MP: np_}[block]
        n_out = {SMG_BLOCK_K: nu + np_, SMG_BLOCK_A: nu, SMG_BLOCK_BT: nu, SMG_BLOCK_B: np_, SMG_BLOCK_MASS: nu,
                 SMG_BLOCK_MP: np_}[block]
        self._check(x, n_in, "x")
        y = self._like(x, n_out) if y is None else y
        self._check(y, n_out, "y")
        _lib.check(self.lib.smg_apply_block(self._h, level, _dtype_code(x), block, _ptr(x), _ptr(y)))
        return y

    def lift_dirichlet(self, level, u_d, b):
        """b <- b - K u~ on free rows, 0 on Dirichlet rows (u~ = u_d on the
        boundary nodes, 0 elsewhere); b updated in place and returned."""
        nu, np_ = self.sizes(level)
        self._check(u_d, nu, "u_d")
        self._check(b, nu + np_, "b")
        if u_d.dtype != b.dtype:
            raise ValueError("u_d and b must have the same dtype")
        _lib.check(self.lib.smg_lift_dirichlet(self._h, level, _dtype_code(b), _ptr(u_d), _ptr(b)))
        return b

    def insert_dirichlet(self, level, u_d, x):
        """x_D <- u_d on the Dirichlet velocity entries; x updated in place."""
        nu, np_ = self.sizes(level)
        self._check(u_d, nu, "u_d")
        self._check(x, nu + np_, "x")
        if u_d.dtype != x.dtype:
            raise ValueError("u_d and x must have the same dtype")
        _lib.check(self.lib.smg_insert_dirichlet(self._h, level, _dtype_code(x), _ptr(u_d), _ptr(x)))
        return x

    def diagonal(self, level, which):
        import torch
        nu, np_ = self.sizes(level)
        out = torch.empty(nu if which == 0 else np_, dtype=torch.float64, device="cuda")
        _lib.check(self.lib.smg_get_diagonal(self._h, level, which, _ptr(out)))
        return out

    def eigs(self, level):
        a, s = ctypes.c_double(), ctypes.c_double()
        _lib.check(self.lib.smg_get_eigs(self._h, level, ctypes.byref(a), ctypes.byref(s)))
        return a.value, s.value

    def set_eigs(self, level, beta_A, beta_S):
        _lib.check(self.lib.smg_set_eigs(self._h, level, float(beta_A), float(beta_S)))

    def chebyshev(self, level, which, r, out=None):
        nu, np_ = self.sizes(level)
        n = nu if which == 0 else np_
        self._check(r, n, "r")
        out = self._like(r, n) if out is None else out
        _lib.check(self.lib.smg_chebyshev(self._h, level, _dtype_code(r), which, _ptr(r), _ptr(out)))
        return out

    def velocity_update(self, level, x, b, uhat=None):
        """uhat = u + sigma Cheb(A, D_A, k_A)(f - A u - B^T p) (the first line
        of an inexact symmetric Uzawa step) for x = (u, p), b = (f, g)."""
        nu, _ = self.sizes(level)
        n = self.n_total(level)
        self._check(x, n, "x")
        self._check(b, n, "b")
        uhat = self._like(x, nu) if uhat is None else uhat
        self._check(uhat, nu, "uhat")
        _lib.check(self.lib.smg_velocity_update(self._h, level, _dtype_code(x), _ptr(x), _ptr(b), _ptr(uhat)))
        return uhat

    def smooth(self, level, x, b, steps=1):
        n = self.n_total(level)
        self._check(x, n, "x")
        self._check(b, n, "b")
        _lib.check(self.lib.smg_smooth(self._h, level, _dtype_code(x), _ptr(x), _ptr(b), int(steps)))
        return x

    def restrict(self, fine_level, r_fine, r_coarse=None):
        self._check(r_fine, self.n_total(fine_level), "r_fine")
        nc = self.n_total(fine_level - 1)
        r_coarse = self._like(r_fine, nc) if r_coarse is None else r_coarse
        self._check(r_coarse, nc, "r_coarse")
        _lib.check(self.lib.smg_restrict(self._h, fine_level, _dtype_code(r_fine), _ptr(r_fine), _ptr(r_coarse)))
        return r_coarse

    def prolongate_add(self, fine_level, w_coarse, x_fine):
        self._check(w_coarse, self.n_total(fine_level - 1), "w_coarse")
        self._check(x_fine, self.n_total(fine_level), "x_fine")
        _lib.check(self.lib.smg_prolongate_add(self._h, fine_level, _dtype_code(x_fine), _ptr(w_coarse), _ptr(x_fine)))
        return x_fine

    def coarse_solve(self, b0, x0=None):
        n = self.n_total(0)
        self._check(b0, n, "b0")
        x0 = self._like(b0, n) if x0 is None else x0
        _lib.check(self.lib.smg_coarse_solve(self._h, _dtype_code(b0), _ptr(b0), _ptr(x0)))
        return x0

    def vcycle(self, level, x, b):
        n = self.n_total(level)
        self._check(x, n, "x")
        self._check(b, n, "b")
        _lib.check(self.lib.smg_vcycle(self._h, level, _dtype_code(x), _ptr(x), _ptr(b)))
        return x

    def _solve(self, fn, x, b, rtol, maxit, raise_on_failure):
        import torch
        n = self.n_total(self.n_levels - 1)
        for t, nm in ((x, "x"), (b, "b")):
            self._check(t, n, nm)
            if t.dtype != torch.float64:
                raise TypeError("solve works on float64 vectors")
        hist = np.zeros(maxit + 2)
        info = _lib.SmgSolveInfo()
        info.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        info.history_capacity = len(hist)
        st = fn(self._h, _ptr(x), _ptr(b), float(rtol), int(maxit), ctypes.byref(info))
        out = {"status": st, "iterations": info.iterations, "rel_residual": info.rel_residual,
               "rate_q": info.rate_q, "t_solve_ms": info.t_solve_ms, "t_setup_ms": info.t_setup_ms,
               "history": hist[:info.history_len].copy()}
        if st != _lib.SMG_OK and raise_on_failure:
            _lib.check(st)
        return out

    def solve(self, x, b, rtol=1e-8, maxit=200, raise_on_failure=True):
        return self._solve(self.lib.smg_solve, x, b, rtol, maxit, raise_on_failure)

    def solve_stationary(self, x, b, rtol=1e-10, maxit=15, raise_on_failure=False):
        return self._solve(self.lib.smg_solve_stationary, x, b, rtol, maxit, raise_on_failure)

    def profile(self, enable=True):
        """Start (or stop) timing every operator-kernel launch with HIP events."""
        _lib.check(self.lib.smg_profile(self._h, 1 if enable else 0))

    def profile_report(self):
        """{key: (count, total_ms, algorithmic_bytes)} of the launches recorded since profile(True)."""
        n = ctypes.c_int64()
        _lib.check(self.lib.smg_profile_report(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        _lib.check(self.lib.smg_profile_report(self._h, buf, n.value + 1, ctypes.byref(n)))
        out = {}
        for line in buf.value.decode().splitlines():
            key, cnt, ms, nbytes = line.rsplit(" ", 3)
            out[key] = (int(cnt), float(ms), float(nbytes))
        return out

    def gradient(self, x, lam, g_logmu=None, g_f=None, want_logmu=True, want_f=True):
        """Adjoint-state gradients (smg_gradient): given the finest-level state x
        and adjoint state lam (float64 GPU vectors), returns (dJ/dlog mu per
        finest cell, dJ/df per velocity DoF); either may be skipped."""
        import torch
        L = self.n_levels - 1
        n = self.n_total(L)
        nu, _ = self.sizes(L)
        for t, nm in ((x, "x"), (lam, "lam")):
            self._check(t, n, nm)
            if t.dtype != torch.float64:
                raise TypeError("gradient works on float64 vectors")
        ncell = int(np.prod(self.cells(L)))
        if want_logmu and g_logmu is None:
            g_logmu = torch.empty(ncell, dtype=torch.float64, device=x.device)
        if want_f and g_f is None:
            g_f = torch.empty(nu, dtype=torch.float64, device=x.device)
        _lib.check(self.lib.smg_gradient(self._h, _ptr(x), _ptr(lam),
                                         _ptr(g_logmu) if want_logmu else None,
                                         _ptr(g_f) if want_f else None))
        return (g_logmu if want_logmu else None), (g_f if want_f else None)

    def pressure_mean_adjoint(self, g):
        """In place on the float64 finest-level vector g: the transpose of the
        pressure normalisation of solve (smg_pressure_mean_adjoint); no-op
        when c_pressure > 0."""
        import torch
        self._check(g, self.n_total(self.n_levels - 1), "g")
        if g.dtype != torch.float64:
            raise TypeError("pressure_mean_adjoint works on float64 vectors")
        _lib.check(self.lib.smg_pressure_mean_adjoint(self._h, _ptr(g)))
        return g

    def cells(self, level):
        """Cells per direction of a level."""
        return [int(c) * 2 ** level for c in list(self.desc.n_coarse)[:self.dim]]

    def node_coordinates(self, level):
        nu, _ = self.sizes(level)
        nv = nu // self.dim
        xyz = np.zeros((nv, self.dim))
        _lib.check(self.lib.smg_node_coordinates(self._h, level, xyz.ctypes.data_as(ctypes.c_void_p)))
        return xyz


class StokesBatch:
    """Independent problems solved together (smg_batch_*): one StokesMG per
    problem, and a batch handle whose cycle and Krylov steps run every
    problem in packed launches (the batched cycle is one graph launch)."""

    def __init__(self, problems, stream=None, solvers=None):
        import torch
        self._b = ctypes.c_void_p()
        self._own = solvers is None
        self.solvers = [StokesMG(**p) for p in problems] if solvers is None else list(solvers)
        self.lib = self.solvers[0].lib
        s = torch.cuda.current_stream().cuda_stream if stream is None else stream
        n = len(self.solvers)
        ctxs = (ctypes.c_void_p * n)(*[m._h.value for m in self.solvers])
        _lib.check(self.lib.smg_batch_create(ctxs, n, ctypes.c_void_p(s), ctypes.byref(self._b)))

    @classmethod
    def from_solvers(cls, solvers, stream=None):
        """A batch over existing StokesMG objects (not closed with the batch)."""
        return cls(None, stream=stream, solvers=solvers)

    def __len__(self):
        return len(self.solvers)

    def _ptrs(self, ts, name):
        import torch
        if len(ts) != len(self.solvers):
            raise ValueError(f"{name}: one vector per problem")
        for m, t in zip(self.solvers, ts):
            m._check(t, m.n_total(m.n_levels - 1), name)
            if t.dtype != torch.float64:
                raise TypeError("batch vectors are float64")
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def solve(self, xs, bs, rtol=1e-8, maxit=300, raise_on_failure=True):
        """Solve every problem (smg_batch_solve); returns the per-problem info dicts."""
        n = len(self.solvers)
        hist = [np.zeros(maxit + 2) for _ in range(n)]
        infos = (_lib.SmgSolveInfo * n)()
        for i in range(n):
            infos[i].history = hist[i].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            infos[i].history_capacity = len(hist[i])
        st = self.lib.smg_batch_solve(self._b, self._ptrs(xs, "x"), self._ptrs(bs, "b"), float(rtol), int(maxit), infos)
        if st != _lib.SMG_OK and raise_on_failure:
            _lib.check(st)
        return [{"iterations": i.iterations, "rel_residual": i.rel_residual, "t_solve_ms": i.t_solve_ms,
                 "t_setup_ms": i.t_setup_ms, "history": hist[k][:i.history_len].copy()}
                for k, i in enumerate(infos)]

    def precondition(self, vs, zs=None):
        """z_i = M_i^-1 v_i for every problem, one graph launch (smg_batch_precondition)."""
        import torch
        zs = [torch.empty_like(v) for v in vs] if zs is None else zs
        _lib.check(self.lib.smg_batch_precondition(self._b, self._ptrs(vs, "v"), self._ptrs(zs, "z")))
        return zs

    def info(self):
        """(packed launches per batched cycle, kernel-variant choice)."""
        nl, var = ctypes.c_int(), ctypes.c_int()
        _lib.check(self.lib.smg_batch_info(self._b, ctypes.byref(nl), ctypes.byref(var)))
        return nl.value, var.value

    def autotune(self, probe_cycles=5):
        """Fastest kernel-variant choice (smg_batch_autotune): (best, [ms per cycle of each choice])."""
        best, n = ctypes.c_int(), ctypes.c_int()
        times = (ctypes.c_double * 16)()
        _lib.check(self.lib.smg_batch_autotune(self._b, int(probe_cycles), ctypes.byref(best), times, ctypes.byref(n)))
        return best.value, [times[i] for i in range(n.value)]

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self.lib.smg_batch_destroy(self._b)
            self._b = ctypes.c_void_p()
        if getattr(self, "_own", False):
            for s in self.solvers:
                s.close()
            self.solvers = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
