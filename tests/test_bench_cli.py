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


def test_default_workload_is_the_learned_mixed_step():
    """The default is the largest single-GPU configuration at the target arithmetic: N = 262144 points
    in d = 64 near an 8-dim subspace, Gaussian h = 1, leaf 1024, mixed precision with the learned
    proposal trained on 2000 blocks of 512 columns x 4096 targets."""
    old = sys.argv
    sys.argv = ["bench.py"]
    try:
        args = bench.parse()
    finally:
        sys.argv = old
    assert args.workload == "learned64" and args.gpus == 1
    w = bench.WORKLOADS["learned64"]
    assert (w["N"], w["d"], w["leaf"], w["h"], w["precision"], w["learned"]) == (262144, 64, 1024, 1.0, "mixed", True)
    assert (w["train_blocks"], w["block_cols"], w["block_rows"]) == (2000, 512, 4096)
    m = bench.WORKLOADS["mixture16"]
    assert (m["N"], m["d"], m["leaf"], m["num_samples"], m["max_rank"], m["tol"]) == (65536, 16, 512, 512, 256, 1e-5)
    assert m["precision"] == "fp64"
    for name in ("separated3", "fmm3"):
        assert bench.WORKLOADS[name]["separation"] > 0
