"""Host-side contract of bench.py (no GPU): one GPU only, and the roofline constants."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_roofline_constants():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.HBM_PEAK_GBS == 8000.0
    # per ray-cell step one FP32 kappa and one FP64 intensity; per ray a 16-byte work item and an
    # 8-byte slot record
    assert bench.BYTES_PER_STEP == 12 and bench.BYTES_PER_RAY == 24
