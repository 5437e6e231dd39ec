"""Host replay of the 3D box-cell operator kernels' memory accesses
(tests/sweep3d_addr_replay.cpp): every block, lane, cell layer and plane of
the column sweep, the cell block and the cell planes, with the kernels' own
address arithmetic (Column3D) and block / chunk decomposition compiled for
the host, checked against the lengths of the vectors they index, for Q2-Q1
and Q3-Q2 on the level shapes of the 64^3 and 32^3 workloads, the parity
meshes (ragged in every direction) and the mesh of the Q3 configuration
whose column-sweep variant faulted once.  CPU only: no kernel is launched."""
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
    exe = str(tmp_path_factory.mktemp("replay") / "sweep3d_addr_replay")
    cmd = [hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-host-only",
           "-I", os.path.join(ROOT, "paper_2205_15770_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "sweep3d_addr_replay.cpp"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


SHAPES = (
    # 64^3 Q2-Q1 hierarchy (6 levels) and 32^3 Q3-Q2 hierarchy (5 levels)
    [(2, (n, n, n)) for n in (2, 4, 8, 16, 32, 64)] + [(3, (n, n, n)) for n in (2, 4, 8, 16, 32)]
    # parity meshes: ragged tiles in every direction
    + [(2, (2, 3, 2)), (2, (4, 6, 4)), (2, (8, 12, 8)), (3, (2, 2, 3)), (3, (4, 4, 6)), (2, (5, 7, 9)), (3, (5, 7, 9))]
)


@pytest.mark.parametrize("k,n", SHAPES)
@pytest.mark.parametrize("waves", [4096, 1, 100000])
def test_every_access_in_bounds(replay, k, n, waves):
    r = subprocess.run([replay, str(k), *map(str, n), str(waves)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    assert r.returncode == 0, r.stdout
    assert " 0 out of bounds" in r.stdout
