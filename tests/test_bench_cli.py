"""bench.py's command line on a host without a GPU run: more than one GPU is
refused with a message (the benchmark measures one GPU), before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_kernel_labels_of_profile_classes():
    """The kernel name bench.py looks up in the traffic summary for each profiled
    class (sweep, dir, epi, group axes, mode), as rocprofv3 prints it."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    w = W.henon_heiles_8d()
    assert bench.kernel_label(w, "c64", (0, 1, 4, 3, 0)) == "k_sweep16<float, 3, true, 4, 3, 0, 8>"
    assert bench.kernel_label(w, "c64", (0, 0, 0, 3, 0)) == "k_sweep16<float, 3, false, 0, -1, 0, 0>"
    assert bench.kernel_label(w, "c128", (3, 0, 1, 1, 1)) == "k_sweep16<double, 1, false, 1, -1, 1, 0>"
    # the three-pass plan: pass B forward / inverse, pass C moments-only / round trip
    assert bench.kernel_label(w, "c64", (1, 0, 0, 3, 3)) == "k_split<float, 0>"
    assert bench.kernel_label(w, "c64", (1, 1, 0, 3, 3)) == "k_split<float, 1>"
    assert bench.kernel_label(w, "c64", (2, 0, 1, 3, 4)) == "k_split<float, 2>"
    assert bench.kernel_label(w, "c64", (2, 1, 0, 3, 3)) == "k_split<float, 3>"
    assert bench.kernel_label(w, "c128", (2, 1, 0, 3, 3)) == "k_split<double, 3>"
    small = W.harmonic_3d()
    assert bench.kernel_label(small, "c128", (0, 0, 1, 3, 0)) == "k_sweep<double>"
