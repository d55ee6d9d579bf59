"""bench.py's command-line contract on the CPU: more than one GPU is refused with a message and a
non-zero status before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""


def test_help_lists_the_workloads():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                         timeout=120, cwd=ROOT)
    assert out.returncode == 0
    for w in ("batch", "dmr", "sphere", "pivots", "sphere-batch"):
        assert w in out.stdout


def test_error_report_names_the_worst_element():
    """bench.py's error statement: per l, max over (r1, r2) of |z - ref| / max |ref_l|, and the
    (l, r1, r2) where the largest one sits."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench

    ref = np.ones((3, 4, 4))
    ref[1] *= 10.0
    z = ref.copy()
    z[2, 1, 3] += 3e-6  # relative to max |ref_2| = 1
    z[1, 0, 0] += 2e-5  # relative to max |ref_1| = 10
    per_l, worst = bench.rel_errors(z, ref)
    assert per_l[0] == 0.0 and abs(per_l[1] - 2e-6) < 1e-12 and abs(per_l[2] - 3e-6) < 1e-12
    assert (worst["l"], worst["r1_bin"], worst["r2_bin"]) == (2, 1, 3)
