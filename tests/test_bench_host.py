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
    # algorithmic bytes: per ray-cell step one FP32 kappa and one FP32 intensity, per ray an
    # 8-byte work item and a 4-byte value; what the kernel moves: a 16-byte cell record per
    # step, an 8-byte work item and an 8-byte slot record per ray
    assert bench.BYTES_PER_STEP == 8 and bench.BYTES_PER_RAY == 12
    assert bench.KERNEL_BYTES_PER_STEP == 16 and bench.KERNEL_BYTES_PER_RAY == 16


def test_default_workload_is_the_dns_size_snapshot():
    sys.path.insert(0, ROOT)
    import bench
    sys.argv = ["bench.py"]
    a = bench.parse()
    assert a.workload == "dns256" and a.gpus == 1 and a.learned_fields >= 5
    from paper_1810_00188_amd import inputs
    w = inputs.dns256()
    assert (w.nx, w.ny, w.nz, w.R, w.kd.nb, w.kd.ng, w.kd.k_dtype, w.march) == (256, 128, 128, 64, 100, 16, "bf16", "f32")
