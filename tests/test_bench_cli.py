"""The benchmark's command-line contract on the CPU: it runs on one GPU only
and refuses more, and the counter-based traffic figure is withheld for
workloads the committed counters do not cover."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus 1" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")          # no JSON line for a refused run


def test_traffic_is_withheld_for_uncovered_workloads():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic("no-such-workload", "f32") is None
    assert bench.measured_traffic(None, "f32") is None
