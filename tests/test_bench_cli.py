"""The benchmark's command-line contract on the CPU: it runs on one GPU only
and refuses more, the counter-based traffic figure is withheld for workloads
the committed counters do not cover, and the open-plane variant's workload
(pure-fluid reservoirs at both x ends, component 1 at the inlet, component 2
at the outlet, no body force) applies to porous samples only."""
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


def test_open_variant_workload():
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    from paper_2207_01534_amd import workloads as wl
    assert bench._open_applies(wl.workload("spheres512", shape=(48, 40, 32)))
    assert not bench._open_applies(wl.workload("droplet32"))                       # no sample
    assert not bench._open_applies(wl.workload("spheres128", shape=(36, 32, 32)))  # too short in x
    w = wl.workload("spheres128", shape=(64, 48, 40))
    wo = wl.open_drainage(w, 10)
    assert (wo.solid[:, :, :10] == 0).all() and (wo.solid[:, :, -10:] == 0).all()
    np.testing.assert_array_equal(wo.solid[:, :, 10:-10], w.solid[:, :, 10:-10])
    assert (wo.xi[wo.solid == 0] == 0).all() and (wo.rho[:, wo.solid != 0] == 0).all()
    assert (wo.rho[0][:, :, :5] > 0.9).all() and (wo.rho[1][:, :, :5] < 0.1).all()     # inlet: component 1
    assert (wo.rho[1][:, :, -10:] > 0.9).all() and (wo.rho[0][:, :, -10:] < 0.1).all()  # outlet: component 2
    assert wo.g == ((0, 0, 0), (0, 0, 0)) and wo.tau == w.tau and wo.G == w.G
