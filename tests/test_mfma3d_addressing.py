"""Host replay of the 3D matrix-core cell kernel's memory accesses
(tests/mfma3d_addr_replay.cpp): every block, lane and cell layer, with the
kernel's own decomposition (mfma3d_chunks, mfma3d_decode) and per-lane
addressing (Mfma3DLane) compiled for the host, checked against the lengths
of the velocity vectors, the viscosity array, the LDS input planes and the
staging area; every velocity node stored by exactly one lane.  Level shapes
of the 64^3 hierarchy and the parity meshes (ragged tiles), with several
z-chunk targets.  CPU only: no kernel is launched."""
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
    exe = str(tmp_path_factory.mktemp("replay") / "mfma3d_addr_replay")
    cmd = [hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-host-only",
           "-I", os.path.join(ROOT, "paper_2205_15770_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "mfma3d_addr_replay.cpp"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


SHAPES = [(n, n, n) for n in (2, 4, 8, 16, 32, 64)] + [(2, 3, 2), (4, 6, 4), (8, 12, 8), (5, 3, 2), (10, 6, 4),
                                                       (20, 12, 8), (33, 17, 5), (1, 1, 1)]


@pytest.mark.parametrize("n", SHAPES)
@pytest.mark.parametrize("waves", [2048, 1, 100000])
def test_every_access_in_bounds(replay, n, waves):
    r = subprocess.run([replay, *map(str, n), str(waves)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    assert r.returncode == 0, r.stdout
    assert " 0 out of bounds" in r.stdout
