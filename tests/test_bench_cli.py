"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a device, and the workload table holds the
configurations the timed step and the parity tests use."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_default_workload_is_the_mixture():
    w = bench.WORKLOADS["mixture16"]
    assert (w["N"], w["d"], w["leaf"], w["num_samples"], w["max_rank"], w["tol"]) == (65536, 16, 512, 512, 256, 1e-5)
    assert w["precision"] == "fp64"
    for name in ("separated3", "fmm3"):
        assert bench.WORKLOADS[name]["separation"] > 0
