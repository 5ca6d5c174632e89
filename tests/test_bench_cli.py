"""Host-side checks of bench.py that need no GPU: the multi-GPU refusal and
the per-call flop count used for the roofline."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_flops_per_call_convention():
    sys.path.insert(0, ROOT)
    import bench
    # N (18 + 43 D): phase 18 per bin, per detector 5 (reduction) + 30 (sin/cos) + 8 (MAC)
    assert bench.flops_per_call(4017, 3) == pytest.approx(4017 * (18 + 43 * 3))
    assert bench.flops_per_call(945, 1) == pytest.approx(945 * 61)
