"""bench.py's host-side contract (no GPU): one GPU only, and the byte model
of the roofline."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sweep_byte_model():
    import bench
    n, m, B = 4_000_000, 70_000_000, 128
    # bf16, over-relaxed: indices 4m, offsets + scales 8n, per node and column 2 (residue read)
    # + 2 (written) + 2 (previous push) + 4 (accumulator read and written every second sweep)
    assert bench.sweep_bytes(n, m, B, True, 2) == 4 * m + 8 * n + 10 * n * B == 5_432_000_000
    # FP32, plain order: 4 + 4 + 4 + 2 (own input residue every second sweep)
    assert bench.sweep_bytes(n, m, B, False, 4) == 4 * m + 8 * n + 14 * n * B
    assert bench.fp64_sweep_bytes(n, m) == 4 * m + 40 * n
