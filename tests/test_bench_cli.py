"""bench.py's host-side contract, without a GPU: more than one GPU is
refused with a message, and the kernel names it looks up in the committed
profiles are the ones the library launches."""
import os
import subprocess
import sys

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, REPO)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(REPO, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_names_and_profiles():
    import bench
    assert bench.kernel_name(3, "mixed", 256) == "k_step_row<Model<3>, float, false, 0>"
    assert bench.kernel_name(3, "fp64", 256) == "k_step<Model<3>, double, false, 0>"
    assert bench.kernel_name(3, "mixed", 100) == "k_step<Model<3>, float, false, 0>"
    assert bench.kernel_name(3, "fp64", 256, "aa_odd") == "k_step<Model<3>, double, false, 3>"
    # whole rows in a 256-cell block: stores rotated through LDS; else stored at x + theta
    assert bench.kernel_name(3, "mixed", 256, "aa_odd") == "k_step_row<Model<3>, float, false, 4>"
    assert bench.kernel_name(3, "mixed", 192, "aa_odd") == "k_step_row<Model<3>, float, false, 2>"
    assert bench.kernel_name(3, "fp64", 5, "aa_odd") == "k_step<Model<3>, double, false, 2>"
    # every committed summary names its kernel, sizes and the sources it was taken of
    prof = os.path.join(REPO, "profiles")
    for name in os.listdir(prof):
        if name.endswith(".txt"):
            text = open(os.path.join(prof, name)).read()
            assert "kernel:" in text and "source_sha256:" in text and "rocprofv3" in text, name
