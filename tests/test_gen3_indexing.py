"""Host replay of the index arithmetic of the 3D general-cell kernels in line
layout (tests/gen3_replay.cpp): division by multiplication against integer
division, every block and lane of the cell kernel (reads inside their
arrays, every per-cell result written exactly once), every thread of the
gather (node coordinates, the cells around a node against brute force,
reads inside the per-cell results), with the kernels' own helpers compiled
for the host, on the level shapes of the 32^3 Q3-Q2 hierarchy and ragged
meshes.  CPU only: no kernel is launched."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("gen3") / "gen3_replay")
    cmd = [hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-host-only",
           "-I", os.path.join(ROOT, "paper_2205_15770_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "gen3_replay.cpp"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


SHAPES = ([(3, (n, n, n)) for n in (2, 4, 8, 16, 32)] + [(2, (n, n, n)) for n in (2, 4, 8, 16)]
          + [(3, (1, 1, 1)), (3, (5, 7, 9)), (3, (2, 2, 3)), (2, (5, 7, 9)), (2, (3, 2, 2)), (3, (9, 3, 2))])


@pytest.mark.parametrize("k,n", SHAPES)
def test_line_kernel_and_gather_indexing(replay, k, n):
    r = subprocess.run([replay, str(k), *map(str, n)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    assert " 0 errors" in r.stdout
