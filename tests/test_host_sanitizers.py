"""The host replays of the 3D kernels' index arithmetic (sweep3d_addr_replay.cpp,
gen3_replay.cpp: the kernels' own decomposition and addressing helpers
compiled for the host) built with AddressSanitizer and UndefinedBehaviorSanitizer
on the host code (-Xarch_host before each -fsanitize=; no GPU code is built),
and run on ragged meshes: no out-of-bounds host access, no signed overflow, no
invalid shift or division in that arithmetic.  CPU only."""
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


def _build(tmp_path_factory, src, name):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("san") / name)
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "-x", "hip", "--offload-host-only",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "paper_2205_15770_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, src), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


@pytest.fixture(scope="module")
def sweep_san(tmp_path_factory):
    return _build(tmp_path_factory, "sweep3d_addr_replay.cpp", "sweep3d_addr_replay_san")


@pytest.fixture(scope="module")
def gen3_san(tmp_path_factory):
    return _build(tmp_path_factory, "gen3_replay.cpp", "gen3_replay_san")


def _run(cmd):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env)


@pytest.mark.parametrize("k,n", [(2, (8, 12, 8)), (2, (5, 7, 9)), (3, (2, 2, 3)), (3, (4, 4, 6))])
def test_sweep_replay_clean_under_sanitizers(sweep_san, k, n):
    r = _run([sweep_san, str(k), *map(str, n), "4096"])
    assert r.returncode == 0, r.stdout
    assert " 0 out of bounds" in r.stdout
    assert "runtime error" not in r.stdout and "AddressSanitizer" not in r.stdout


@pytest.mark.parametrize("k,n", [(3, (5, 7, 9)), (2, (3, 2, 2)), (3, (8, 8, 8))])
def test_gen3_replay_clean_under_sanitizers(gen3_san, k, n):
    r = _run([gen3_san, str(k), *map(str, n)])
    assert r.returncode == 0, r.stdout
    assert " 0 errors" in r.stdout
    assert "runtime error" not in r.stdout and "AddressSanitizer" not in r.stdout
