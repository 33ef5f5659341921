"""Host-side checks of bench.py (no GPU): the one-GPU guard and the
algorithmic flop counts the roofline uses."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_flop_counts():
    import bench
    # 32 n^3 with n = ceil(N/2): 4 N^3 for even N
    assert bench.flops_per_slice_step(240) == 4 * 240 ** 3
    assert bench.flops_per_slice_step(480) == 4 * 480 ** 3
    assert bench.flops_per_slice_step(121) == 32 * 61 ** 3
    assert abs(bench.dense_equiv_flops(240) - 1.060e8) / 1.060e8 < 1e-3
