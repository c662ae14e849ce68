"""The committed counter summaries (no GPU needed).  bench.py reports a
kernel's HBM traffic only while the sha256 of its sources matches the hash
stored with the counters; where it matches, the stored bytes must be those of
the kernel's fields."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    try:
        import bench as b
    finally:
        sys.path.remove(ROOT)
    return b


@pytest.mark.parametrize("nel", [1024, 4096])
def test_traffic_matches_current_sources(bench, nel):
    ndof = (nel + 2) ** 2
    w = 4   # FP32
    alg = {"assemble_s1_fuel": 4 * w * ndof, "assemble_s3": 3 * w * ndof,
           "sweep_x_A": 2 * w * ndof, "sweep_y_M": 2 * w * ndof, "sweep_y_cn": 2 * w * ndof}
    for kernel, a in alg.items():
        t = bench.measured_traffic(kernel, nel)
        if t is None:
            pytest.skip(f"{kernel} at {nel}^2: counters predate the kernel's sources "
                        "(bench.py reports its traffic as null)")
        # at least the algorithmic bytes of a whole field, at most twice them
        assert 0.4 * a < t < 2.0 * a, (kernel, nel, t / a)


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(os.path.join(ROOT, "profiles"))
                                        if f.endswith(".md")))
def test_summaries_state_their_command(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert "rocprofv3" in text and "bench.py" in text
    assert len(text) < 16384   # short summaries, not raw output
