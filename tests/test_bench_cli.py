"""bench.py's command line on a machine without a GPU: more than one GPU is refused with a message
and exit status 2, before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_only_selects_known_legs():
    sys.path.insert(0, ROOT)
    import bench
    argv = sys.argv
    try:
        sys.argv = ["bench.py", "--only", "massive_onlattice"]
        a = bench.parse()
    finally:
        sys.argv = argv
    assert not a.no_onlattice and a.no_variants and a.no_adjoint and a.no_batch and a.no_forcing and a.no_3d
    assert a.no_staged_large
    try:
        sys.argv = ["bench.py", "--only", "staged_large"]
        a = bench.parse()
    finally:
        sys.argv = argv
    assert not a.no_staged_large and a.no_onlattice and a.no_variants and a.no_adjoint and a.no_3d
