"""bench.py runs on one GPU only: asking for more exits with status 2 and a
message, before generating inputs or touching a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_measured_traffic_only_for_its_sources_and_shape():
    sys.path.insert(0, ROOT)
    import bench
    m = bench.MEASURED_TRAFFIC
    for shape, b in m["bytes_per_launch"].items():
        # within a few percent of the algorithmic bytes of one pass (28 B per stored point)
        assert 1.0 <= b / (28 * 32082542) < 1.05
        if bench.kpass_sources_sha256() == m["sources_sha256"]:
            assert bench.measured_traffic(shape) == b
        else:
            assert bench.measured_traffic(shape) is None
    assert bench.measured_traffic((1, 1, 1)) is None
