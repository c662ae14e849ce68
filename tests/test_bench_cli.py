"""bench.py's command line, without a GPU: more than one GPU is refused with a
message before anything touches a device, and the defaults are one GPU and
a bounded number of steps."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_defaults(monkeypatch):
    sys.path.insert(0, ROOT)
    try:
        import bench
        monkeypatch.setattr(sys, "argv", ["bench.py"])
        a = bench.parse()
    finally:
        sys.path.remove(ROOT)
    assert a.gpus == 1 and a.steps == 200 and a.warmup == 20 and a.nel == 1024
    assert not (a.no_ensembles or a.no_paper_meshes or a.no_other_schemes or a.no_cpu_baseline)
