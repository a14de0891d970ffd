"""Benchmark of the coupled LBM + dynamic-IB step on one MI355X.

Default workload: the symmetric Y-bifurcation (main diameter D = 32, daughters
0.8 D at 60 degrees, fillet 4, 256x128x40 grid, Re = 10, tau = 0.7) with one
deformable 2562-vertex capsule (occlusion 0.5, Ca = 0.01), populations in
FP32.  A particle-free precursor run (untimed) develops the flow before the
capsule is released, then W warm-up steps and K timed steps are run from a
captured HIP graph.  Prints one JSON line.

Metric: lattice updates per second of the full coupled step, counted on the
fluid (non-solid) nodes; the box-node rate is reported alongside.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "MLUPS (D3Q19 LBM+IB step), % HBM roofline; batched & adjoint vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fluid_kernel_traffic.json")
# sources that decide what the fluid kernels read and write (code and launch shapes)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2207_06043_amd", "csrc", n)
               for n in ("lbm_kernels.hip", "lbm_abi.cpp", "lbm_internal.h")]
FLUID_KERNELS = ("k_fluid_all", "k_fluid_bulk", "k_fluid_rec")


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the fused stream-collide kernel from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source; else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}:{precision}")
    if not e or e.get("kernel_sha") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def _counter_medians(run_dir, counter):
    """Median per-dispatch value (KiB) of a rocprofv3 --pmc counter for each
    kernel name in run_dir/run_counter_collection.csv."""
    import csv
    import statistics
    vals = {}
    with open(os.path.join(run_dir, "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: statistics.median(v) for k, v in vals.items()}


def summarize_counters(args):
    """Writes the HBM traffic of one launch of the fluid kernels (bulk +
    boundary records, the span the roofline times) into TRAFFIC_FILE, from
    FETCH_SIZE and WRITE_SIZE runs of the workload and of the plain-copy
    calibration (--copy-calibration-mb), each scaled so the copy reads and
    writes its known size."""
    wl_f, wl_w, cp_f, cp_w = args.summarize_counters
    copy_bytes = args.calibration_bytes

    def only(d, key):
        hits = [v for k, v in d.items() if key in k]
        if len(hits) != 1:
            raise SystemExit(f"expected one kernel matching {key}, found {len(hits)}")
        return hits[0]

    kf = copy_bytes / (only(_counter_medians(cp_f, "FETCH_SIZE"), "copyBuffer") * 1024.0)
    kw = copy_bytes / (only(_counter_medians(cp_w, "WRITE_SIZE"), "copyBuffer") * 1024.0)
    fetch = _counter_medians(wl_f, "FETCH_SIZE")
    write = _counter_medians(wl_w, "WRITE_SIZE")
    rd = sum(1024.0 * kf * v for k, v in fetch.items() if any(n in k for n in FLUID_KERNELS))
    wr = sum(1024.0 * kw * v for k, v in write.items() if any(n in k for n in FLUID_KERNELS))
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        d = {}
    d[f"{args.workload}:{args.precision}"] = {
        "kernel_sha": kernel_hash(),
        "bytes_per_launch": round(rd + wr),
        "read_bytes": round(rd),
        "write_bytes": round(wr),
        "fetch_scale": round(kf, 5),
        "write_scale": round(kw, 5),
        "kernels": {k: {"FETCH_SIZE_KiB": fetch.get(k), "WRITE_SIZE_KiB": write.get(k)}
                    for k in sorted(set(fetch) | set(write)) if any(n in k for n in FLUID_KERNELS)},
    }
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(d[f"{args.workload}:{args.precision}"]))


def build_workload(name, precision):
    import synth
    if name == "bifurcation_capsule":
        return synth.bifurcation_capsule(precision=precision)
    if name == "pipe_sphere":
        return synth.pipe_sphere(precision=precision)
    if name == "periodic_r0":
        return synth.periodic_r0(precision=precision)
    if name == "pipe_r1":
        return synth.pipe_r1(precision=precision)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, target_s=15.0):
    """The FP64 oracle as it stands, on the host cores, on a bounded sample of
    the same workload (the first steps after release)."""
    import oracle
    t0 = time.time()
    sim = oracle.from_workload(w)
    setup = time.time() - t0
    t = time.time()
    sim.step(2)
    per = (time.time() - t) / 2
    n = max(2, min(2000, int(target_s / max(per, 1e-6))))
    t = time.time()
    sim.step(n)
    dt = time.time() - t
    nf = w.domain.n_fluid
    return {"value": round(nf * n / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.lib().orc_threads(),
            "kind": "oracle",
            "sample": f"{w.name}: {n} coupled steps (after 2 untimed) of the same grid and capsule, "
                      f"FP64, {dt:.1f} s (+{setup:.1f} s setup), lattice updates counted on fluid nodes"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="bifurcation_capsule")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--precursor", type=int, default=2000,
                    help="particle-free steps before the capsule is released (untimed)")
    ap.add_argument("--kernel-steps", type=int, default=500,
                    help="steps whose fused stream-collide launches are timed with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration-mb", type=float, default=0.0,
                    help="only run plain device copies of this size (calibrates HBM counters)")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR",
                    "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="turn rocprofv3 --pmc runs into the fluid-kernel traffic entry (no GPU)")
    ap.add_argument("--calibration-bytes", type=float, default=1.024e9,
                    help="bytes read and written by one calibration copy")
    args = ap.parse_args()
    if args.summarize_counters:
        args.precision = args.precision or ("f64" if args.workload == "pipe_sphere" else "f32")
        summarize_counters(args)
        return
    if args.copy_calibration_mb > 0:
        import torch
        n = int(args.copy_calibration_mb * 1e6 / 4)
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the build has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2207_06043_amd as P

    precision = args.precision or ("f64" if args.workload == "pipe_sphere" else "f32")
    w = build_workload(args.workload, precision)
    torch.cuda.set_device(0)
    lat = P.Lattice(w.domain, w.tau, w.u_max, precision)
    if args.precursor > 0 and w.bodies:
        lat.step(args.precursor)
        lat.sync()
    for b in w.bodies:
        lat.add_body(b)
    info = lat.info()
    lat.step(args.warmup)
    lat.sync()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    status = lat.sync(raise_on_stop=False)
    if status != P.LBM_OK:
        print(json.dumps({"metric": METRIC, "error": f"device stopped with status {status} "
                          "inside the timed region: throughput invalid"}))
        sys.exit(1)
    elapsed = t1 - t0
    n_fluid, n_box = info["n_fluid"], info["n_nodes"]
    value = n_fluid * args.steps / elapsed / 1e6

    # fused stream-collide kernel: average launch duration from HIP events
    avg_ms = lat.time_fluid_kernel(args.kernel_steps)
    status = lat.sync(raise_on_stop=False)
    bytes_alg = info["bytes_per_step_alg"]
    achieved = bytes_alg / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, precision)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precision,
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "grid": [w.domain.nx, w.domain.ny, w.domain.nz],
            "fluid_nodes": n_fluid,
            "box_nodes": n_box,
            "bodies": len(w.bodies),
            "vertices": info["n_vertices"],
            "lups_counted_on": "fluid nodes",
            "mlups_box": round(n_box * args.steps / elapsed / 1e6, 2),
            "markers_per_s": round(info["n_faces"] * 3 * args.steps / elapsed, 1) if w.bodies else 0,
            "precursor_steps": args.precursor if w.bodies else 0,
            "parallelism": "single GPU",
            "cache_note": "working set %.1f MB fits the 256 MB Infinity Cache" % (bytes_alg / 1e6)
            if bytes_alg < 200e6 else "working set exceeds the Infinity Cache",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_fluid_all (fused pull-stream + bounce-back + Zou-He + forced BGK collide, "
                       "boundary records and bulk tiles in one launch)" if info["fluid_launch"] == 1 else
                       "k_fluid_bulk || k_fluid_rec (fused pull-stream + BCs + forced BGK collide, "
                       "bulk tiles and boundary records on two streams)"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch_alg": bytes_alg,
            "avg_launch_us": round(avg_ms * 1e3, 3),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
