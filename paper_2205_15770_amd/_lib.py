"""ctypes binding of libsmg.so (include/smg.h): argument marshalling only.

Every entry point takes device pointers (torch tensors on the GPU are passed
by data_ptr()); all arithmetic runs in the HIP kernels of the library.  The
binding raises if the library is missing: there is no CPU fallback."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmg.so")

SMG_OK, SMG_EINVAL, SMG_ENOMEM, SMG_EDEVICE, SMG_ENOTCONV, SMG_EBREAKDOWN, SMG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SMG_F64, SMG_F32 = 0, 1
SMG_SCHUR_D, SMG_SCHUR_LOC, SMG_SCHUR_P, SMG_SCHUR_EXACT = 0, 1, 2, 3
SMG_FORM_GRAD, SMG_FORM_EPS = 0, 1
SMG_BLOCK_K, SMG_BLOCK_A, SMG_BLOCK_BT, SMG_BLOCK_B, SMG_BLOCK_MASS, SMG_BLOCK_MP = 0, 1, 2, 3, 4, 5
SMG_PRECOND_F64, SMG_PRECOND_F32 = 0, 1

STATUS_NAMES = {0: "SMG_OK", -1: "SMG_EINVAL", -2: "SMG_ENOMEM", -3: "SMG_EDEVICE",
                -4: "SMG_ENOTCONV", -5: "SMG_EBREAKDOWN", -6: "SMG_EUNSUPPORTED"}

EXPORTS = ["smg_desc_default", "smg_create", "smg_destroy", "smg_sizes", "smg_set_stream",
           "smg_vmult", "smg_vmult_noalloc", "smg_residual", "smg_apply_block", "smg_lift_dirichlet", "smg_insert_dirichlet", "smg_get_diagonal", "smg_get_eigs",
           "smg_set_eigs", "smg_chebyshev", "smg_velocity_update", "smg_smooth", "smg_restrict", "smg_prolongate_add",
           "smg_coarse_solve", "smg_vcycle", "smg_solve", "smg_solve_stationary", "smg_batch_create",
           "smg_batch_destroy", "smg_batch_solve", "smg_batch_precondition", "smg_batch_info", "smg_batch_autotune",
           "smg_node_coordinates", "smg_gradient", "smg_pressure_mean_adjoint", "smg_profile", "smg_profile_report",
           "smg_last_error"]


class SmgDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("fe_degree", ctypes.c_int),
                ("n_coarse", ctypes.c_int * 3), ("n_levels", ctypes.c_int),
                ("box_lo", ctypes.c_double * 3), ("box_hi", ctypes.c_double * 3),
                ("fine_vertices", ctypes.POINTER(ctypes.c_double)),
                ("mu", ctypes.c_double), ("mu_cell", ctypes.POINTER(ctypes.c_double)),
                ("gamma", ctypes.c_double), ("rho", ctypes.c_double), ("c_pressure", ctypes.c_double),
                ("cheb_deg_A", ctypes.c_int), ("cheb_deg_S", ctypes.c_int),
                ("smooth_steps", ctypes.c_int), ("cycle_index", ctypes.c_int),
                ("schur_diag", ctypes.c_int), ("precision", ctypes.c_int),
                ("fgmres_restart", ctypes.c_int), ("stream", ctypes.c_void_p), ("form", ctypes.c_int)]


class SmgSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("rate_q", ctypes.c_double), ("t_solve_ms", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_capacity", ctypes.c_int),
                ("history_len", ctypes.c_int)]


class SmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load libsmg.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with paper_2205_15770_amd.build.build()")
    lib = ctypes.CDLL(path)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, None
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "smg_desc_default": (V, [ctypes.POINTER(SmgDesc)]),
        "smg_create": (I, [ctypes.POINTER(SmgDesc), ctypes.POINTER(P)]),
        "smg_destroy": (I, [P]),
        "smg_sizes": (I, [P, I, i64p, i64p]),
        "smg_set_stream": (I, [P, P]),
        "smg_vmult": (I, [P, I, I, P, P]),
        "smg_vmult_noalloc": (I, [P, I, I, P, P]),
        "smg_residual": (I, [P, I, I, P, P, P]),
        "smg_apply_block": (I, [P, I, I, I, P, P]),
        "smg_lift_dirichlet": (I, [P, I, I, P, P]),
        "smg_insert_dirichlet": (I, [P, I, I, P, P]),
        "smg_get_diagonal": (I, [P, I, I, P]),
        "smg_get_eigs": (I, [P, I, dp, dp]),
        "smg_set_eigs": (I, [P, I, D, D]),
        "smg_chebyshev": (I, [P, I, I, I, P, P]),
        "smg_velocity_update": (I, [P, I, I, P, P, P]),
        "smg_smooth": (I, [P, I, I, P, P, I]),
        "smg_restrict": (I, [P, I, I, P, P]),
        "smg_prolongate_add": (I, [P, I, I, P, P]),
        "smg_coarse_solve": (I, [P, I, P, P]),
        "smg_vcycle": (I, [P, I, I, P, P]),
        "smg_solve": (I, [P, P, P, D, I, ctypes.POINTER(SmgSolveInfo)]),
        "smg_solve_stationary": (I, [P, P, P, D, I, ctypes.POINTER(SmgSolveInfo)]),
        "smg_batch_create": (I, [ctypes.POINTER(P), I, P, ctypes.POINTER(P)]),
        "smg_batch_destroy": (I, [P]),
        "smg_batch_solve": (I, [P, ctypes.POINTER(P), ctypes.POINTER(P), D, I, ctypes.POINTER(SmgSolveInfo)]),
        "smg_batch_precondition": (I, [P, ctypes.POINTER(P), ctypes.POINTER(P)]),
        "smg_batch_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "smg_batch_autotune": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(I)]),
        "smg_node_coordinates": (I, [P, I, P]),
        "smg_gradient": (I, [P, P, P, P, P]),
        "smg_pressure_mean_adjoint": (I, [P, P]),
        "smg_profile": (I, [P, I]),
        "smg_profile_report": (I, [P, ctypes.c_char_p, ctypes.c_int64, i64p]),
        "smg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error():
    return load().smg_last_error().decode()


def check(status):
    if status != SMG_OK:
        raise SmgError(status, last_error())
    return status
