"""The benchmark's command-line contract on the CPU: one GPU only (a clear
exit for more), and the oracle's CPU-baseline leg on the small workload."""
import os
import subprocess
import sys

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_cpu_baseline_times_the_oracle():
    sys.path.insert(0, ROOT)
    import bench
    out = bench.cpu_baseline([W.TINY], None, 60.0)
    assert out["kind"] == "oracle" and out["unit"] == "solves/s"
    assert out["value"] > 0 and "bound" not in out
    assert "n=1600" in out["sample"] and out["cores"] >= 1
    # a sample that cannot finish is reported as an upper bound
    big = bench.cpu_baseline(W.batch_params()[:1], None, 1.0)
    assert big["bound"] == "upper" and abs(big["value"] - 1.0) < 1e-12 and big["cores"] >= 1


def test_studies_command_line_needs_a_device():
    """The Fig. 2/4/5 studies run through the device library; without a HIP
    device the command line says so and exits with status 2."""
    import torch
    if torch.cuda.is_available():
        return
    r = subprocess.run([sys.executable, "-m", "paper_1411_4356_amd.studies", "rcm", "--nc", "2", "--nm", "4"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2 and "HIP device" in r.stderr
