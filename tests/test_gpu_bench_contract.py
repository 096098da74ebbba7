"""The benchmark's output contract on the GPU: one JSON line with the
throughput, the roofline of the dominant kernel and the oracle's host
baseline, on the small droplet workload (a few seconds); and the open-plane
variant on a small sphere pack."""
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_complete_json_line(monkeypatch, capsys):
    sys.path.insert(0, ROOT)
    import bench
    argv = ["bench.py", "--workload", "droplet32", "--steps", "20", "--warmup", "4", "--cpu-seconds", "1",
            "--no-adjoint"]
    print("[case] " + " ".join(argv), flush=True)
    capsys.readouterr()
    monkeypatch.setattr(sys, "argv", argv)
    bench.main()
    out = capsys.readouterr().out
    lines = [l for l in out.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 4 and d["higher_is_better"] is True
    assert d["value"] > 0 and d["unit"] == "MLUPS" and d["dtype"] == "f32"
    assert "workload" in d["config"]
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-3)
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
    assert cb["one_core_value"] > 0 and "cpu_model" in cb
    assert set(d["variants"]) == {"f16", "bf16"}


def test_bench_open_plane_variant(monkeypatch, capsys):
    sys.path.insert(0, ROOT)
    import bench
    argv = ["bench.py", "--workload", "spheres128", "--shape", "64,64,64", "--steps", "20", "--warmup", "4",
            "--no-cpu-baseline", "--no-adjoint", "--variants", "open"]
    print("[case] " + " ".join(argv), flush=True)
    capsys.readouterr()
    monkeypatch.setattr(sys, "argv", argv)
    bench.main()
    out = capsys.readouterr().out
    d = json.loads([l for l in out.splitlines() if l.strip()][-1])
    v = d["variants"]["open"]
    assert v["mlups"] > 0 and v["nonfinite"] == 0
    o = v["open_x"]
    assert o["rho1_in"] == bench.OPEN_RHO[0] and o["rho2_out"] == bench.OPEN_RHO[1]
    assert o["periodic_ms_per_step"] > 0 and o["fluid_nodes"] > d["config"]["fluid_nodes"]
    assert v["collide_stream_traffic_gbs"] is None
