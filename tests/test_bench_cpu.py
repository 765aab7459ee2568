"""bench.py's contract on the host: more than one GPU is refused with a
message and exit status 2 before any GPU work, and the algorithmic work
figures it reports are defined from the oracle's counters."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_flop_weights_and_peaks():
    sys.path.insert(0, ROOT)
    import bench
    # the roofline's weights: candidate distance 9, side test 6, new vertex 12, fan tetrahedron 28
    assert bench.FLOP_WEIGHTS == dict(candidates=9, vertex_tests=6, new_vertices=12, fan_triangles=28)
    assert bench.FP64_VECTOR_PEAK == 78.6e12 and bench.HBM_PEAK == 8.0e12
    # the committed counter summary is read only while the kernel sources match it
    assert bench.committed_traffic("no such kernel") is None
