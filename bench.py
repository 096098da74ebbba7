#!/usr/bin/env python3
"""Throughput benchmark of the two-component D3Q19 pseudopotential step on one MI355X.

A step is one pass of the whole hot path over the lattice: densities,
virtual solid densities (IVSD), forces, forced SRT collision and streaming
with bounce-back, all in the HIP kernels of libmclbm.so.  The default
workload is the 512^3 sphere pack (radius 12, porosity ~0.38), single-buffer
streaming, FP32 storage; the FP16 and BF16 offset-storage forms, and the FP32
step with open inlet/outlet planes along x (the drainage drive of Sec. 4.1, on
the same pack with 10-plane fluid reservoirs at both x ends, timed open and
periodic), are timed in the same run and reported under "variants".

Prints one JSON line.  ``value`` is MLUPS over all lattice nodes (solid
included) with the state resident in HBM; the roofline object prices the
dominant kernel (forces + collision + streaming) against the 8 TB/s HBM peak
using its algorithmic bytes (populations read + written per fluid node plus
one mask byte per node) and its average duration from HIP events recorded on
the library's stream over the timed region.  The FP64 oracle is timed on the
host cores on a bounded sub-block of the same workload (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & HBM GB/s (2-comp D3Q19), FP32 vs FP16-storage; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
POP_BYTES = {"f32": 2 * 19 * 2 * 4,                 # 304 B per fluid node
             "f16": 2 * (18 * 2 + 4) * 2,           # 160 B: 36 FP16 moving + 2 FP32 rest
             "bf16": 2 * (18 * 2 + 4) * 2}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def describe(w):
    return (f"{w.name}: {w.shape[0]}x{w.shape[1]}x{w.shape[2]} "
            + ("periodic droplet" if w.name.startswith("droplet") else "synthetic porous medium")
            + f", tau=({w.tau[0]}, {w.tau[1]}), G={w.G}, porosity {w.n_fluid / w.n_nodes:.4f}")


# Open-plane variant: component 1 imposed at the inlet slightly above the bulk
# density it takes at G = 3.5 (about 1.05), component 2 at the outlet at it.
OPEN_RHO = (1.07, 1.05)
OPEN_RESERVOIR = 10


def _open_applies(w):
    """The open-plane variant runs on porous samples long enough in x for two
    reservoirs and the sample between them."""
    return bool((w.solid != 0).any()) and w.shape[0] >= 4 * OPEN_RESERVOIR


def run_gpu(w, storage, steps, warmup, open_x=None):
    import torch
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams, Storage
    st = {"f32": Storage.F32, "f16": Storage.F16, "bf16": Storage.BF16}[storage]
    p = LatticeParams(shape=w.shape, tau=w.tau, G=w.G, g=w.g, storage=st, fluid_capacity=w.n_fluid)
    lat = Lattice(p, torch.as_tensor(w.solid), torch.as_tensor(w.xi),
                  torch.as_tensor(w.rho.astype(np.float32)))
    if open_x is not None:
        lat.set_open_x(*open_x)
    lat.step(warmup)
    torch.cuda.synchronize()
    lat.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = lat.profile_read()
    lat.profile(False)
    # the same number of steps without the per-kernel events (on small
    # lattices, whose kernels last microseconds, the event records dominate)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t1
    diag = lat.diagnostics(raise_nonfinite=False)
    n, nf = w.n_nodes, w.n_fluid
    k2_ms, k2_n = prof["collide_stream"]
    k2_avg_s = k2_ms / 1e3 / max(k2_n, 1)
    k2_bytes = nf * POP_BYTES[storage] + n * 1
    res = {
        "mlups": n * steps / dt / 1e6,
        "mlups_without_events": n * steps / dt_plain / 1e6,
        "mflups": nf * steps / dt / 1e6,
        "ms_per_step": dt / steps * 1e3,
        "gbs_alg_step": (nf * POP_BYTES[storage] + n) * steps / dt / 1e9,
        "kernels_ms_avg": {k: (v[0] / max(v[1], 1)) for k, v in prof.items()},
        "collide_stream_bytes_per_launch": k2_bytes,
        "collide_stream_gbs": k2_bytes / k2_avg_s / 1e9,
        "mass": [diag["mass1"], diag["mass2"]],
        "nonfinite": diag["nonfinite"],
    }
    del lat
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def adjoint_cases():
    """The adjoint cost cases: (label, workload, initial densities, region or
    None for the trapped region of the unperturbed run).
      adjoint64           64^3 pack r = 6, xi ~ U[-0.4, 0.4], non-wetting phase in
                          the inlet buffers, loss over the sample interior;
      adjoint64_trapped   the same pack with the non-wetting phase seeded as
                          twelve ganglia of radius 4 (seed 6403), loss over the
                          ganglia still trapped after the forward run;
      adjoint128          the 128^3 pack r = 8 with xi ~ U[-0.4, 0.4] (seed 6401),
                          a state of 2.8e2 MB that lives in HBM, not in the
                          last-level cache, loss over the sample interior."""
    from paper_2207_01534_amd import workloads as wl

    def interior(shape):
        nx, ny, nz = shape
        region = np.zeros((nz, ny, nx), np.uint8)
        region[:, :, 3:nx - 3] = 1
        return region

    w64 = wl.workload("adjoint64")
    w128 = wl.workload("spheres128")
    w128.xi = wl.uniform_xi(w128.solid, -0.4, 0.4, seed=6401)
    return [("adjoint64: 64^3 sphere pack r=6, porosity 0.40, xi~U[-0.4,0.4], loss over the sample interior",
             w64, w64.rho, interior(w64.shape)),
            ("adjoint64_trapped: the 64^3 pack with 12 non-wetting ganglia r=4, loss over the trapped ganglia",
             w64, wl.ganglia_rho(w64.solid, 12, 4.0, seed=6403), None),
            ("adjoint128: 128^3 sphere pack r=8, porosity 0.40, xi~U[-0.4,0.4], loss over the sample interior",
             w128, w128.rho, interior(w128.shape))]


def run_adjoint(label, w, rho0, region, steps=500, every=25):
    """Adjoint cost of one case: forward, forward with checkpoints, and the
    reverse sweep (segment recompute included), median of three after one
    untimed pass of each.  The checkpoint buffer also holds the level log
    (every level's pseudopotential field and the last segment's states), so
    that the segment recompute runs the collide-stream kernel only and skips
    the last segment; the same sweep without the log is timed too, and the
    two gradients compared bit for bit.  region None: the
    trapped non-wetting region of the unperturbed forward run
    (workloads.trapped_region), then frozen."""
    import torch
    from paper_2207_01534_amd import workloads as wl
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams
    rho = torch.as_tensor(rho0.astype(np.float32), device="cuda")
    lat = Lattice(LatticeParams(shape=w.shape, tau=w.tau, G=w.G, g=w.g), torch.as_tensor(w.solid),
                  torch.as_tensor(w.xi), rho)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def median_of(fn, reps=3):
        runs = [timed(fn) for _ in range(reps)]
        runs.sort(key=lambda r: r[1])
        return runs[reps // 2]

    def forward():
        lat.init_equilibrium(rho)
        return lat.step(steps)

    def forward_checkpointed(level_log=True):
        lat.init_equilibrium(rho)
        return lat.step_checkpointed(steps, every, level_log=level_log)

    # warm-up: one pass of each timed operation (clocks, code objects, work buffer)
    forward()
    if region is None:
        region = wl.trapped_region(lat.density().cpu().numpy(), w.solid)
    reg = torch.as_tensor(region, device="cuda")
    ck = forward_checkpointed()
    lat.gradient_snw(steps, every, ck, reg)
    _, t_fwd = median_of(forward)
    _, t_fwd_ck = median_of(forward_checkpointed)
    ck = forward_checkpointed()  # the reverse sweep differentiates the latest recording
    grad, t_bwd = median_of(lambda: lat.gradient_snw(steps, every, ck, reg))
    # the same without the level log: the recompute also forms each level's psi-hat
    del ck
    ck = forward_checkpointed(level_log=False)
    lat.gradient_snw(steps, every, ck, reg)
    grad0, t_bwd0 = median_of(lambda: lat.gradient_snw(steps, every, ck, reg))
    out = {"workload": label, "steps": steps, "every": every, "region_voxels": int(region.sum()),
           "forward_ms": t_fwd * 1e3, "forward_checkpointed_ms": t_fwd_ck * 1e3, "backward_ms": t_bwd * 1e3,
           "cost_ratio": t_bwd / t_fwd, "cost_ratio_vs_checkpointed": t_bwd / t_fwd_ck,
           "level_log": True, "backward_without_level_log_ms": t_bwd0 * 1e3,
           "cost_ratio_without_level_log": t_bwd0 / t_fwd,
           "gradients_bitwise_equal": bool(torch.equal(grad, grad0)),
           "boundary_voxels": lat.boundary_count(), "grad_abs_max": float(grad.abs().max())}
    del lat, ck, grad, grad0
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


# everything that decides what the step kernels touch: the kernels, their
# launchers and the workspace layout (plane stride, skew) set by the C ABI
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2207_01534_amd", "csrc", f)
                  for f in ("lbm_device.hpp", "lbm_tiles.hpp", "lbm_kernels.hpp", "lbm_kernels.hip",
                            "mclbm_api.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_step_kernels.json")
CODEC = {"f32": "CodecF32", "f16": "CodecF16", "bf16": "CodecBF16"}


def measured_traffic(workload_name, storage):
    """HBM bytes per collide-stream launch (odd and even launches alternate, so
    the mean of the two instantiations) from the committed rocprofv3 counter
    summary, or None when it does not cover this workload/storage or the kernel
    sources changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    h = hashlib.sha256(b"".join(open(p, "rb").read() for p in KERNEL_SOURCES)).hexdigest()
    per = rec["workloads"].get(workload_name, {}).get(storage, {})
    ks = [v for k, v in per.items() if k.startswith(f"k_collide_stream<{CODEC[storage]},")]
    if rec.get("kernel_source_sha256") != h or len(ks) != 2:
        return None
    return sum(v["read_bytes"] + v["write_bytes"] for v in ks) / len(ks)


def cpu_baseline(w, target_s):
    """FP64 oracle on a bounded sub-block of the workload (periodic sub-lattice)."""
    # every CPU this process may run on, unless the environment already fixes
    # the OpenMP thread count (a machine's CPU share per GPU)
    os.environ.setdefault("OMP_NUM_THREADS", str(len(os.sched_getaffinity(0))))
    from oracle import oracle as orc
    nx, ny, nz = w.shape
    sx, sy, sz = min(nx, 256), min(ny, 128), min(nz, 128)
    solid = np.ascontiguousarray(w.solid[:sz, :sy, :sx])
    xi = np.ascontiguousarray(w.xi[:sz, :sy, :sx]).astype(np.float64)
    rho = np.ascontiguousarray(w.rho[:, :sz, :sy, :sx]).astype(np.float32).astype(np.float64)
    o = orc.Oracle(orc.OracleParams((sx, sy, sz), tau=w.tau, G=w.G, g=w.g), solid, xi)
    o.init_equilibrium(rho)
    t0 = time.perf_counter()
    o.run(1)
    one = time.perf_counter() - t0
    k = max(1, int(round(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    o.run(k)
    dt = time.perf_counter() - t0
    n = sx * sy * sz
    cores = orc.num_threads()
    # per-core rate: the same sub-block on one thread, a few seconds of work
    orc.set_num_threads(1)
    t0 = time.perf_counter()
    o.run(1)
    one1 = time.perf_counter() - t0
    k1 = max(1, min(k, int(target_s / 4.0 / max(one1, 1e-3))))
    t0 = time.perf_counter()
    o.run(k1)
    dt1 = time.perf_counter() - t0
    orc.set_num_threads(cores)
    return {"value": n * k / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{sx}x{sy}x{sz} sub-block of {w.name} (periodic), {k} FP64 steps in {dt:.1f} s",
            "one_core_value": n * k1 / dt1 / 1e6,
            "one_core_sample": f"same sub-block on 1 thread, {k1} steps in {dt1:.1f} s",
            "cpu_model": _cpu_model(), "visible_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def _cpu_model():
    """The model string of /proc/cpuinfo with its family/model/stepping numbers
    (a virtual machine may report only a short model name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (t.strip() for t in line.split(":", 1))
                if k in ("model name", "vendor_id", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                    info[k] = v
            if not line.strip() and info:
                break
    except OSError:
        return None
    if not info:
        return None
    return (f"{info.get('model name', '?')} ({info.get('vendor_id', '?')}, family {info.get('cpu family', '?')}, "
            f"model {info.get('model', '?')}, stepping {info.get('stepping', '?')}, {info.get('cpu MHz', '?')} MHz)")


def calibrate_copy():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch, 3 launches.
    The byte counters a profiler reports for it give the scale for the step kernels."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}))


def copy_bandwidth(reps=10):
    """Achievable HBM bandwidth on this GPU: a plain elementwise copy, 1 GiB read
    + 1 GiB written per launch (far beyond the last-level cache), timed with
    HIP events on the current stream; GB/s of the median launch."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        torch.neg(a, out=b)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.neg(a, out=b)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    times.sort()
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 4 / times[reps // 2] / 1e9


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="spheres512")
    ap.add_argument("--shape", default=None, help="override the workload's shape, e.g. 512,512,512")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--variants", default="f16,bf16,open",
                    help="extra forms timed in the same run: storage forms and 'open' (FP32 with "
                         "open x planes); comma list, '' for none")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost measurement")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB elementwise copy (reference for HBM byte counters)")
    ap.add_argument("--adjoint-only", default=None, metavar="CASES",
                    help="only time the named adjoint cases (comma list of adjoint64, adjoint64_trapped, "
                         "adjoint128) and print their records, one JSON line each")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.adjoint_only:
        wanted = [c for c in args.adjoint_only.split(",") if c]
        for label, w_a, rho_a, region_a in adjoint_cases():
            if label.split(":")[0] in wanted:
                _log(f"timing the adjoint ({label.split(':')[0]}, 500 steps, checkpoint every 25)")
                print(json.dumps(run_adjoint(label, w_a, rho_a, region_a)), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the step is a single-GPU kernel path in this "
              "project (multi-GPU z-slab decomposition is a design, not built); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    from paper_2207_01534_amd import workloads as wl
    t0 = time.perf_counter()
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    w = wl.workload(args.workload, shape=shape)
    _log(f"workload {args.workload} built in {time.perf_counter() - t0:.1f}s; "
         f"nodes {w.n_nodes} fluid {w.n_fluid}")

    _log(f"timing {args.storage}: warmup {args.warmup}, steps {args.steps}")
    main_res = run_gpu(w, args.storage, args.steps, args.warmup)
    _log(f"{args.storage}: {main_res['mlups']:.0f} MLUPS")
    variants = {}
    for v in [s for s in args.variants.split(",") if s and s != args.storage]:
        if v not in POP_BYTES and v != "open":
            ap.error(f"unknown variant {v!r}")
        _log(f"timing variant {v}")
        if v == "open":
            if not _open_applies(w):
                _log("open: skipped (not a porous sample with room for the reservoirs)")
                continue
            wo = wl.open_drainage(w, OPEN_RESERVOIR)
            variants[v] = run_gpu(wo, "f32", args.steps, args.warmup, open_x=OPEN_RHO)
            periodic = run_gpu(wo, "f32", args.steps, args.warmup)
            variants[v]["open_x"] = {
                "rho1_in": OPEN_RHO[0], "rho2_out": OPEN_RHO[1], "reservoir_planes": OPEN_RESERVOIR,
                "fluid_nodes": wo.n_fluid, "body_force": 0.0,
                "periodic_ms_per_step": round(periodic["ms_per_step"], 4),
                "extra_ms_per_step": round(variants[v]["ms_per_step"] - periodic["ms_per_step"], 4)}
        else:
            variants[v] = run_gpu(w, v, args.steps, args.warmup)
        _log(f"{v}: {variants[v]['mlups']:.0f} MLUPS")

    adjoint = None
    if not args.no_adjoint:
        cases = []
        for label, w_a, rho_a, region_a in adjoint_cases():
            _log(f"timing the adjoint ({label.split(':')[0]}, 500 steps, checkpoint every 25)")
            cases.append(run_adjoint(label, w_a, rho_a, region_a))
            _log(f"adjoint {label.split(':')[0]}: backward/forward = {cases[-1]['cost_ratio']:.2f}")
        # the first case keeps the top-level keys; every case is listed
        adjoint = dict(cases[0])
        adjoint["cases"] = cases

    cpu = None
    if not args.no_cpu_baseline:
        _log("timing the FP64 oracle on a host sub-block")
        cpu = cpu_baseline(w, args.cpu_seconds)
        _log(f"oracle: {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")

    k2 = main_res["collide_stream_gbs"]
    name = w.name if not args.shape else None
    copy_gbs = copy_bandwidth()
    _log(f"plain copy: {copy_gbs:.0f} GB/s")

    def traffic_of(res, storage):
        if storage not in POP_BYTES:
            return None, None
        t = measured_traffic(name, storage)
        ms = res["kernels_ms_avg"]["collide_stream"]
        return t, (round(t / (ms * 1e-3) / 1e9, 1) if t else None)

    traffic, traffic_gbs = traffic_of(main_res, args.storage)
    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded sphere pack standing in for the paper's rock images)",
        "config": {"workload": describe(w), "storage": args.storage, "shape": list(w.shape),
                   "nodes": w.n_nodes, "fluid_nodes": w.n_fluid, "streaming": "single-buffer AA"},
        "roofline": {"bound": "hbm", "achieved": round(k2, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(k2 / HBM_PEAK_GBS, 4),
                     "traffic": round(traffic) if traffic else None,
                     "traffic_gbs": traffic_gbs,
                     "kernel": "k_collide_stream",
                     "algorithmic_bytes_per_launch": main_res["collide_stream_bytes_per_launch"],
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(k2 / copy_gbs, 4),
                     "traffic_frac_of_copy": round(traffic_gbs / copy_gbs, 4) if traffic_gbs else None},
        "cpu_baseline": cpu,
        "mlups_without_events": round(main_res["mlups_without_events"], 1),
        "mflups": round(main_res["mflups"], 1),
        "gbs_alg_step": round(main_res["gbs_alg_step"], 1),
        "kernels_ms_avg": {k: round(v, 4) for k, v in main_res["kernels_ms_avg"].items()},
        "adjoint": adjoint,
        "variants": {k: {"mlups": round(v["mlups"], 1), "mlups_without_events": round(v["mlups_without_events"], 1),
                         "mflups": round(v["mflups"], 1),
                         "ms_per_step": round(v["ms_per_step"], 4),
                         "gbs_alg_step": round(v["gbs_alg_step"], 1),
                         "collide_stream_gbs": round(v["collide_stream_gbs"], 1),
                         "collide_stream_traffic_gbs": traffic_of(v, k)[1],
                         "nonfinite": v["nonfinite"],
                         "kernels_ms_avg": {kk: round(vv, 4) for kk, vv in v["kernels_ms_avg"].items()},
                         **({"open_x": v["open_x"]} if "open_x" in v else {})}
                     for k, v in variants.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
