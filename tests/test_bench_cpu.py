"""bench.py's host-side contract, no GPU: more than one GPU is refused with a
message, and the energy counter reports why it is unavailable instead of
failing when no GPU counter can be read."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_energy_counter_unavailable_without_gpu():
    sys.path.insert(0, ROOT)
    import bench
    import torch
    if torch.cuda.is_available():
        return  # the GPU tests exercise the counter through the benchmark itself
    read, why = bench.energy_counter()
    assert read is None and isinstance(why, str) and why
