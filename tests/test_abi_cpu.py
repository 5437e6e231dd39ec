"""C ABI checks that need no GPU: the library loads, exports every function
include/smg.h declares, fills defaults, and rejects invalid descriptors and
arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smg.h")
LIB = os.path.join(ROOT, "paper_2205_15770_amd", "libsmg.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsmg.so not built (run __graft_entry__.build())")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smg_[a-z_]+)\s*\(", text)))


def test_header_declarations_are_exported():
    from paper_2205_15770_amd import _lib
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == names


def test_desc_default_values():
    from paper_2205_15770_amd import _lib
    lib = _lib.load()
    d = _lib.SmgDesc()
    lib.smg_desc_default(ctypes.byref(d))
    assert (d.dim, d.fe_degree, d.n_levels) == (2, 2, 3)
    assert list(d.n_coarse) == [4, 4, 4]
    assert (d.cheb_deg_A, d.cheb_deg_S, d.smooth_steps, d.cycle_index) == (1, 1, 2, 1)
    assert d.mu == 1.0 and d.rho == 1.0 and d.gamma == 0.0 and d.c_pressure == 0.0
    assert d.fgmres_restart == 30
    assert d.form == _lib.SMG_FORM_GRAD and d.schur_diag == _lib.SMG_SCHUR_D


@pytest.mark.parametrize("field,value,code", [
    ("dim", 4, -1), ("fe_degree", 1, -1), ("fe_degree", 4, -6), ("n_levels", 1, -1),
    ("smooth_steps", 0, -1), ("cycle_index", 3, -1), ("schur_diag", 5, -1), ("precision", 7, -1),
    ("fgmres_restart", 0, -1), ("cheb_deg_A", -1, -1), ("gamma", -1.0, -1), ("mu", 0.0, -1),
    ("rho", 0.0, -1), ("c_pressure", -0.5, -1), ("schur_diag", 4, -1), ("form", 2, -1),
])
def test_invalid_descriptors_rejected_without_device(field, value, code):
    from paper_2205_15770_amd import _lib
    lib = _lib.load()
    d = _lib.SmgDesc()
    lib.smg_desc_default(ctypes.byref(d))
    setattr(d, field, value)
    h = ctypes.c_void_p(1234)
    st = lib.smg_create(ctypes.byref(d), ctypes.byref(h))
    assert st == code
    assert h.value is None
    assert len(lib.smg_last_error()) > 0


def test_coarse_mesh_condition_and_box():
    from paper_2205_15770_amd import _lib
    lib = _lib.load()
    d = _lib.SmgDesc()
    lib.smg_desc_default(ctypes.byref(d))
    d.n_coarse[1] = 1          # a coarse cell with two opposite boundary faces (App. A)
    h = ctypes.c_void_p()
    assert lib.smg_create(ctypes.byref(d), ctypes.byref(h)) == -1
    lib.smg_desc_default(ctypes.byref(d))
    d.box_hi[0] = d.box_lo[0]
    assert lib.smg_create(ctypes.byref(d), ctypes.byref(h)) == -1


def test_null_arguments_rejected():
    from paper_2205_15770_amd import _lib
    lib = _lib.load()
    assert lib.smg_create(None, None) == -1
    assert lib.smg_vmult(None, 0, 0, None, None) == -1
    assert lib.smg_sizes(None, 0, None, None) == -1
    assert lib.smg_solve(None, None, None, 1e-8, 10, None) == -1
    assert lib.smg_destroy(None) == 0
    assert b"null" in lib.smg_last_error() or lib.smg_last_error() == b""


def test_unsupported_combinations_rejected_without_device():
    from paper_2205_15770_amd import _lib
    lib = _lib.load()
    d = _lib.SmgDesc()
    lib.smg_desc_default(ctypes.byref(d))
    d.form = _lib.SMG_FORM_EPS
    d.schur_diag = _lib.SMG_SCHUR_LOC        # built for the gradient form only
    h = ctypes.c_void_p()
    assert lib.smg_create(ctypes.byref(d), ctypes.byref(h)) == -6
    assert h.value is None


def test_dirichlet_entry_points_reject_null_arguments():
    from paper_2205_15770_amd import _lib
    lib = _lib.load()
    assert lib.smg_lift_dirichlet(None, 0, 0, None, None) == -1
    assert lib.smg_insert_dirichlet(None, 0, 0, None, None) == -1



def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a header struct, from a C program built with
    the host compiler against include/smg.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "layout.c"
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "smg.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    out = subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True, check=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("struct,cls", [("smg_desc", "SmgDesc"), ("smg_solve_info", "SmgSolveInfo")])
def test_binding_structs_match_the_header(struct, cls, tmp_path):
    """The ctypes mirrors of the header's structs (t_setup_ms among the solve
    fields) have the C layout: size and every field's offset."""
    from paper_2205_15770_amd import _lib
    c = getattr(_lib, cls)
    fields = [f for f, _ in c._fields_]
    size, offs = _c_layout(struct, fields, tmp_path)
    assert ctypes.sizeof(c) == size
    assert [getattr(c, f).offset for f in fields] == offs
