"""Host-side contract of bench.py (no GPU): more than one GPU is refused with
a JSON message, and the workload table matches the sizes the line reports."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_default_workload_sizes():
    sys.path.insert(0, ROOT)
    import bench
    wl = bench.WORKLOADS["stokes2d_q2q1_512"]
    n = [c * 2 ** (wl["n_levels"] - 1) for c in wl["n_coarse"]]
    assert n == [512, 512]
    k = wl["fe_degree"]
    # velocity 2 (k n + 1)^2, pressure ((k - 1) n + 1)^2: the 2,364,419 DoFs of the record
    assert 2 * (k * 512 + 1) ** 2 + ((k - 1) * 512 + 1) ** 2 == 2364419
