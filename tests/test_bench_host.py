"""Host checks of bench.py's contract pieces: one GPU only, the committed
counter summary matching the kernel sources (so the reported HBM traffic is
the current kernel's), and the counted operations per face."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_summary_matches_kernel_sources():
    """The face kernels' HBM bytes come from profiles/ only while the source
    hash recorded there is the current one; a kernel change without new
    counters makes this fail instead of reporting stale traffic."""
    for d in range(3):
        t = bench.measured_traffic(f"k_face<3, 3, {d}, double, false, false, false>")
        assert t is not None and 5e9 < t < 1e10, (d, t)


def test_counted_operations_per_face():
    ops = bench.load_ops()
    for k in ("face_x", "face_y", "face_z"):
        assert 1000 < ops[k] < 5000, ops
