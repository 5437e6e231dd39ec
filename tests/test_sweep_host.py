"""Host-side checks of the parameter-study module: its problem sizes are the
paper's DoF counts (Sec. 4: 2467 and 148 739 DoFs for the 2D examples, 2312
and 112 724 for the 3D cavity), computed from the Q2-Q1 lattice sizes."""
import numpy as np

from paper_2205_15770_amd.sweep import CASES


def _dofs(dim, n):
    return dim * (2 * n + 1) ** dim + (n + 1) ** dim


def test_case_sizes_match_the_paper():
    want = {"laser": (2467, 148739), "cavity2d": (2467, 148739), "cavity3d": (2312, 112724)}
    for name, c in CASES.items():
        n0 = c["n_coarse"][0]
        assert all(v == n0 for v in c["n_coarse"])
        small = _dofs(c["dim"], n0 * 2 ** (c["small_levels"] - 1))
        large = _dofs(c["dim"], n0 * 2 ** (c["large_levels"] - 1))
        assert (small, large) == want[name]
