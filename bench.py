"""Benchmark of the coupled LBM + dynamic-IB step on one MI355X.

Default workload: the symmetric Y-bifurcation (main diameter D = 32, daughters
0.8 D at 60 degrees, fillet 4, 256x128x40 grid, Re = 10, tau = 0.7) with one
deformable 2562-vertex capsule (occlusion 0.5, Ca = 0.01), populations in
FP32.  A particle-free precursor run (untimed) develops the flow before the
capsule is released, then W warm-up steps and K timed steps are run from a
captured HIP graph.  Prints one JSON line.

Metric: lattice updates per second of the full coupled step, counted on the
fluid (non-solid) nodes; the box-node rate is reported alongside.

Other workloads: ``--workload precision_form`` (512x256x64 bifurcation with
16 capsules, FP16 storage by default), ``--workload batch_instances`` (the
batching form: 64 bifurcations of uneven size advanced together, tuned, and
compared with the same instances stepped one by one), ``--workload
differentiation_form`` (the coupled adjoint sweep with the capsule against the
plain steps), ``--workload capsule_train`` (trains of three capsules, soft or
with rigid spheres, ``--train``/``--junction``), ``pipe_sphere`` and the
bandwidth workloads ``periodic_r0`` and ``pipe_r1``.  With ``--log-out`` the
released steps run as a logged run (surface strain, centre, Taylor
deformation and stretch of every body every ``--log-every`` steps, up to the
damage stop) and the log is written to that file.
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
FLUID_KERNELS = ("k_fluid_all", "k_fluid_bulk", "k_fluid_rec", "kb_fluid_all", "kb_fluid_bulk",
                 "kb_fluid_rec")


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic_key(workload, precision, shape=None):
    key = f"{workload}:{precision}"
    if shape:
        key += ":" + ",".join(str(shape[k]) for k in ("bulk_v", "block", "mode", "per_xcd"))
    return key


def measured_traffic(workload, precision, shape=None):
    """HBM bytes per launch of the fused stream-collide kernel (the batched
    fluid phase for the batching form, keyed by its launch shape) from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source; else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = d.get(traffic_key(workload, precision, shape))
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


def _counter_totals(run_dir, counter):
    """Sum over all dispatches (KiB) of a rocprofv3 --pmc counter for each
    kernel name in run_dir/run_counter_collection.csv."""
    import csv
    tot = {}
    with open(os.path.join(run_dir, "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                tot[r["Kernel_Name"]] = tot.get(r["Kernel_Name"], 0.0) + float(r["Counter_Value"])
    return tot


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
    if args.workload == "differentiation_form":
        # every dispatch of the sweep's kernels, per adjoint step of the run
        # (the warmup call and the timed call)
        names, per = ADJ_KERNELS, 1.0 / (args.warmup + args.steps)
        fetch = _counter_totals(wl_f, "FETCH_SIZE")
        write = _counter_totals(wl_w, "WRITE_SIZE")
    else:
        names, per = FLUID_KERNELS, 1.0
        fetch = _counter_medians(wl_f, "FETCH_SIZE")
        write = _counter_medians(wl_w, "WRITE_SIZE")
    rd = per * sum(1024.0 * kf * v for k, v in fetch.items() if any(n in k for n in names))
    wr = per * sum(1024.0 * kw * v for k, v in write.items() if any(n in k for n in names))
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        d = {}
    shape = None
    if args.batch_shape:
        shape = dict(zip(("bulk_v", "block", "mode", "per_xcd"), map(int, args.batch_shape.split(","))))
    key = traffic_key(args.workload, args.precision, shape)
    d[key] = {
        "kernel_sha": kernel_hash(),
        "bytes_per_launch": round(rd + wr),
        "read_bytes": round(rd),
        "write_bytes": round(wr),
        "fetch_scale": round(kf, 5),
        "write_scale": round(kw, 5),
        "kernels": {k: {"FETCH_SIZE_KiB": fetch.get(k), "WRITE_SIZE_KiB": write.get(k)}
                    for k in sorted(set(fetch) | set(write)) if any(n in k for n in names)},
    }
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(d[key]))


def build_workload(name, precision, train="soft", junction="smooth"):
    import synth
    if name == "capsule_train":
        return synth.capsule_train(train, precision=precision, junction=junction)
    if name == "bifurcation_capsule":
        return synth.bifurcation_capsule(precision=precision)
    if name == "pipe_sphere":
        return synth.pipe_sphere(precision=precision)
    if name == "periodic_r0":
        return synth.periodic_r0(precision=precision)
    if name == "pipe_r1":
        return synth.pipe_r1(precision=precision)
    if name == "precision_form":
        return synth.precision_form(precision=precision)
    raise SystemExit(f"unknown workload {name}")


def default_precision(workload):
    return {"pipe_sphere": "f64", "precision_form": "f16s"}.get(workload, "f32")


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s=15.0):
    """The FP64 oracle as it stands, on the host cores, on a bounded sample of
    the same workload (its first steps, from the workload's start, restarted
    from there when the sample is longer than the workload's own run); then
    the same with one thread, on a shorter sample."""
    import oracle

    def run(n):
        """Seconds of stepping (set-up excluded) for n steps of w."""
        done, dt = 0, 0.0
        while done < n:
            sim = oracle.from_workload(w)
            k = min(n - done, max(1, w.steps))
            t = time.time()
            st = sim.step(k)
            dt += time.time() - t
            if st != 0:
                raise SystemExit(f"oracle stopped with status {st} in the CPU sample of {w.name}")
            done += k
        return dt

    t0 = time.time()
    oracle.from_workload(w)
    setup = time.time() - t0
    per = run(2) / 2
    n = max(2, min(2000, int(target_s / max(per, 1e-6))))
    dt = run(n)
    nf = w.domain.n_fluid
    threads = oracle.lib().orc_threads()
    oracle.lib().orc_set_threads(1)
    try:
        per1 = run(1)
        n1 = max(1, min(500, int(target_s / 3 / max(per1, 1e-6))))
        dt1 = run(n1)
    finally:
        oracle.lib().orc_set_threads(0)
    restarts = "" if n <= w.steps else f", restarted from the start every {w.steps} steps"
    return {"value": round(nf * n / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "value_1_thread": round(nf * n1 / dt1 / 1e6, 3), "cpu_model": cpu_model(),
            "sample": f"{w.name}: {n} steps of the same grid and bodies on {threads} threads{restarts}, "
                      f"FP64, {dt:.1f} s (+{setup:.1f} s set-up per start); then {n1} steps on 1 thread, "
                      f"{dt1:.1f} s; lattice updates counted on fluid nodes"}


def measured_copy_gbs(nbytes=1.024e9, reps=10):
    """Bandwidth of a plain device-to-device copy of nbytes (read + write
    bytes over the time of reps copies, HIP events): the achievable figure
    beside the datasheet peak."""
    import torch
    n = int(nbytes / 4)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(gbs, 1)


def cpu_baseline_batch(ws, target_s=15.0):
    """The FP64 oracle on a seeded subset (the first 8 instances), each for
    an equal share of the time budget."""
    import oracle
    sub = ws[:8]
    tot_updates, tot_time, steps = 0, 0.0, []
    for w in sub:
        sim = oracle.from_workload(w)
        t = time.time()
        sim.step(1)
        per = time.time() - t
        n = max(1, int(target_s / len(sub) / max(per, 1e-6)))
        t = time.time()
        sim.step(n)
        tot_time += time.time() - t
        tot_updates += w.domain.n_fluid * n
        steps.append(n)
        del sim
    return {"value": round(tot_updates / tot_time / 1e6, 3), "unit": "MLUPS",
            "cores": oracle.lib().orc_threads(), "kind": "oracle",
            "sample": f"instances 0-{len(sub) - 1} of the batching form, {steps} coupled steps each "
                      f"(after 1 untimed), FP64, {tot_time:.1f} s, lattice updates counted on fluid nodes"}


def run_batch(args):
    """The batching form: the instances advance together (one launch per
    phase, graph replay) after the autotuner has picked the fluid launch
    shape; then the same instances are stepped one by one with their own
    step for the comparison."""
    import torch
    import paper_2207_06043_amd as P
    import synth
    precision = args.precision or "f32"
    ws = synth.batch_instances(n_instances=args.instances, workers=min(16, os.cpu_count() or 1))
    for w in ws:
        w.precision = precision
    torch.cuda.set_device(0)
    lats = [P.from_workload(w, precision=precision) for w in ws]
    infos = [lat.info() for lat in lats]
    batch = P.Batch(lats)
    if args.batch_shape:
        batch.set_shape(*map(int, args.batch_shape.split(",")))
        tried = []
    else:
        tried = batch.tune(reps=args.tune_reps)
    shape = batch.shape()
    batch.step(args.warmup)
    for lat in lats:
        lat.sync(raise_on_stop=False)
    done0 = [lat.info()["steps_done"] for lat in lats]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stopped = [k for k, lat in enumerate(lats) if lat.sync(raise_on_stop=False) != P.LBM_OK]
    done = [lat.info()["steps_done"] - d0 for lat, d0 in zip(lats, done0)]
    elapsed = t1 - t0
    n_fluid = sum(i["n_fluid"] for i in infos)
    n_box = sum(i["n_nodes"] for i in infos)
    # an instance that stopped (a damaged capsule) does no more work: only the
    # updates actually performed are counted
    updates = sum(i["n_fluid"] * d for i, d in zip(infos, done))
    value = updates / elapsed / 1e6
    avg_ms = batch.time_fluid(args.kernel_reps)
    bytes_alg = sum(i["bytes_per_step_alg"] for i in infos)
    achieved = bytes_alg / (avg_ms * 1e-3) / 1e9
    # the same instances, one by one, with their own step
    plain, bad = float("nan"), []
    if args.plain_steps > 0:
        for lat in lats:
            lat.sync(raise_on_stop=False)
        done1 = [lat.info()["steps_done"] for lat in lats]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for lat in lats:
            lat.step(args.plain_steps)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        bad = [k for k, lat in enumerate(lats) if lat.sync(raise_on_stop=False) != P.LBM_OK]
        upd_plain = sum(i["n_fluid"] * (lat.info()["steps_done"] - d1)
                        for i, lat, d1 in zip(infos, lats, done1))
        plain = upd_plain / (t3 - t2) / 1e6
    fluid_kernel = ("kb_fluid_all (records and bulk tiles of all instances in one launch)"
                    if shape["mode"] == 0 else
                    "kb_fluid_rec then kb_fluid_bulk (records, then bulk tiles, of all instances)"
                    + (f", persistent bulk grid of {shape['per_xcd']} blocks per XCD"
                       if shape["per_xcd"] else ""))
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
            "workload": "batch_instances",
            "instances": len(ws),
            "fluid_nodes": n_fluid,
            "box_nodes": n_box,
            "bodies": sum(len(w.bodies) for w in ws),
            "vertices": sum(i["n_vertices"] for i in infos),
            "lups_counted_on": "fluid nodes",
            "mlups_box": round(n_box * args.steps / elapsed / 1e6, 2),
            "tuned_shape": shape,
            "shapes_tried": len(tried),
            "plain_one_by_one_mlups": round(plain, 2) if plain == plain else None,
            "plain_steps_each": args.plain_steps,
            "batched_vs_plain": round(value / plain, 3) if plain == plain else None,
            "plain_stopped": bad,
            "instances_stopped": {str(k): done[k] for k in stopped},
            "updates_counted": "fluid nodes x steps each instance actually completed",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": fluid_kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("batch_instances", precision, shape),
            "bytes_per_launch_alg": bytes_alg,
            "avg_launch_us": round(avg_ms * 1e3, 3),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(ws, args.cpu_seconds)
    print(json.dumps(out))


ADJ_KERNELS = ("k_adj_", "k_adjb_", "k_taylor")


def adj_bytes_per_step(n_fluid, n_records, n_w, s):
    """Algorithmic bytes of one adjoint step with states stored in s bytes
    per population: per fluid node, the forward pass and the segment
    recompute (each a pull and a write of 19 populations, 2 x 2 x 19 s), the
    step back (reads the pulled populations, 19 s, and the next step's mu at
    the neighbours, writes mu: 2 x 152 B; two mask words, 8 B); per node
    where the observable w is non-zero, its 152 B; per boundary record, its
    populations entering the collision kept by the recompute and read back
    (2 x 152 B)."""
    return n_fluid * (4 * 19 * s + 19 * s + 2 * 152 + 8) + n_w * 152 + n_records * 2 * 152


def run_adjoint(args):
    """The differentiation form: the bifurcation of the single-capsule case
    (256x128x40, D = 32) after its particle-free precursor, with the
    2562-vertex capsule released; one call of the coupled adjoint over
    args.steps steps with checkpoints every args.checkpoint_every steps
    (states in the lattice's precision, FP32 unless --precision f64; the
    adjoint in FP64) gives the gradients of the time-integrated Taylor
    deformation of the capsule plus the upper daughter's flux with respect to
    the inlet-velocity scale, the body force, the relaxation time and the
    membrane stiffness; then the same number of plain coupled steps of the
    same lattice for the comparison."""
    import torch
    import numpy as np
    import paper_2207_06043_amd as P
    import synth
    w = synth.bifurcation_capsule(precision="f64")
    d = w.domain
    torch.cuda.set_device(0)
    precision = args.precision or "f32"
    lat = P.Lattice(d, w.tau, w.u_max, precision)
    if args.precursor > 0:
        lat.step(args.precursor)
        lat.sync()
    lat.add_body(w.bodies[0])
    info = lat.info()
    n_fluid, n_box = info["n_fluid"], info["n_nodes"]
    out_nodes = np.flatnonzero(d.node_type == synth.OUTLET)
    up = out_nodes[(out_nodes // d.nx) % d.ny == d.ny - 1]
    e_y = torch.tensor([0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1], dtype=torch.float64)
    wv = torch.zeros(19, d.n_nodes, dtype=torch.float64)
    wv[:, torch.from_numpy(up)] = e_y[:, None]
    wv = wv.cuda()
    K = args.checkpoint_every
    if args.warmup > 0:
        lat.adjoint_run(args.warmup, None, wv, taylor_weight=1.0, checkpoint_every=K)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(lat.stream)
    lam, grad, _, J = lat.adjoint_run(args.steps, None, wv, taylor_weight=1.0, checkpoint_every=K)
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    gpu_s = ev0.elapsed_time(ev1) * 1e-3
    value = n_fluid * args.steps / elapsed / 1e6
    # the same number of plain coupled steps of the same lattice
    lat.step(args.warmup)
    lat.sync()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lat.step(args.steps)
    lat.sync()
    torch.cuda.synchronize()
    plain = n_fluid * args.steps / (time.perf_counter() - t2) / 1e6
    bytes_step = adj_bytes_per_step(n_fluid, info["n_general"], len(up), 8 if precision == "f64" else 4)
    achieved = bytes_step / (gpu_s / args.steps) / 1e9
    g = grad.cpu().numpy()
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
        "dtype": precision + " forward, f64 adjoint",
        "data": "synthetic",
        "config": {
            "workload": "differentiation_form",
            "grid": [d.nx, d.ny, d.nz],
            "fluid_nodes": n_fluid,
            "box_nodes": n_box,
            "bodies": 1,
            "vertices": info["n_vertices"],
            "precursor_steps": args.precursor,
            "checkpoint_every": K,
            "objective": ("sum over the steps of the capsule's Taylor deformation plus the upper daughter's "
                          "outward flux; gradient w.r.t. inlet-velocity scale, body force, relaxation time "
                          "and membrane-stiffness scale"),
            "J": [float(J[0]), float(J[1])],
            "lups_counted_on": "fluid nodes x adjoint steps (forward pass, recompute and reverse step included)",
            "plain_mlups": round(plain, 2),
            "adjoint_vs_plain": round(value / plain, 4),
            "grad": [float(x) for x in g],
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("one coupled adjoint step: the fluid step back (k_adj_reverse_all, twice: force "
                       "adjoint at the forced nodes, then the whole step) with the forward-pass, recompute "
                       "and re-run launches of k_adj_fwd_all, and the IB transposes (k_adjb_*)"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("differentiation_form", precision),
            "bytes_per_step_alg": bytes_step,
            "avg_step_us": round(gpu_s / args.steps * 1e6, 3),
            "peak_copy_measured": measured_copy_gbs(),
        },
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, args.cpu_seconds)
        cb["sample"] += ("; forward coupled steps only (from rest): a central-difference derivative "
                         "costs two such runs per parameter")
        out["cpu_baseline"] = cb
    print(json.dumps(out))


def run_logged(args, lat, w, info, precision):
    """The released steps as a logged run (campaign.log_run): the surface
    strain dS(t) = S/S0 - 1, centre, Taylor deformation and largest stretch
    of every body every --log-every steps against t u_max / D, up to the
    damage stop; the log goes to --log-out, the line reports the throughput
    of the logged run (recording included)."""
    import torch
    import paper_2207_06043_amd as P
    D = 2.0 * w.domain.meta["params"]["R"] if "params" in w.domain.meta else 1.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    log = P.campaign.log_run(lat, args.steps, args.log_every, w.u_max, D)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log.update({"workload": w.name, "precision": precision, "grid": [w.domain.nx, w.domain.ny, w.domain.nz],
                "D": D, "u_max": w.u_max, "precursor_steps": args.precursor, "every": args.log_every,
                "bodies": log["bodies"],
                "kinds": ["rigid" if b.rigid else "soft" for b in w.bodies]})
    with open(args.log_out, "w") as f:
        json.dump(log, f)
    n_fluid = info["n_fluid"]
    done = max(log["steps_done"], 1)
    out = {"metric": METRIC, "value": round(n_fluid * done / elapsed / 1e6, 2), "unit": "MLUPS", "n_gpus": 1,
           "steps": done, "warmup": 0, "ms_per_step": round(elapsed / done * 1e3, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": precision, "data": "synthetic",
           "config": {"workload": w.name, "logged_run": True, "log": args.log_out, "status": log["status"],
                      "peak_dS": [b["peak_dS"] for b in log["bodies"]],
                      "t_peak": [b["t_peak"] for b in log["bodies"]],
                      "fluid_nodes": n_fluid, "bodies": len(w.bodies), "parallelism": "single GPU"}}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's run length less the warm-up)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="bifurcation_capsule")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--precursor", type=int, default=None,
                    help="particle-free steps before the capsules are released (untimed; "
                         "default 2000, 1000 for precision_form)")
    ap.add_argument("--kernel-steps", type=int, default=500,
                    help="steps whose fused stream-collide launches are timed with HIP events")
    ap.add_argument("--instances", type=int, default=64, help="batch_instances: how many")
    ap.add_argument("--tune-reps", type=int, default=5, help="batch_instances: timed launches per shape")
    ap.add_argument("--kernel-reps", type=int, default=50,
                    help="batch_instances: timed launches of the tuned fluid phase")
    ap.add_argument("--batch-shape", default=None,
                    help="batch_instances: fluid launch shape 'V,block,mode,per_xcd' instead of tuning")
    ap.add_argument("--plain-steps", type=int, default=32,
                    help="batch_instances: steps of each instance alone for the comparison")
    ap.add_argument("--checkpoint-every", type=int, default=100,
                    help="differentiation_form: checkpoint interval of the adjoint sweep")
    ap.add_argument("--train", default="soft", help="capsule_train: soft, rigid_top, rigid_middle, "
                    "rigid_bottom or all_rigid")
    ap.add_argument("--junction", default="smooth", help="capsule_train: smooth or sharp")
    ap.add_argument("--log-every", type=int, default=100,
                    help="with --log-out: steps between records of the surface strain dS(t)")
    ap.add_argument("--log-out", default=None,
                    help="bodies: run the released steps as a logged run (dS, centre, Taylor deformation, "
                         "stretch every --log-every steps, up to the damage stop) and write the log here")
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
        args.precision = args.precision or default_precision(args.workload)
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

    # run lengths of the workloads: the bifurcation capsule 5000 steps after a
    # 2000-step precursor, the precision form 2000 steps after a 1000-step
    # precursor, the batching form 1000 steps, the pipe with the rigid sphere
    # its 200 steps from the developed Poiseuille flow (the sphere would leave
    # the 48-node pipe in a longer run)
    lengths = {"precision_form": (1000, 100, 1900), "batch_instances": (0, 50, 950),
               "differentiation_form": (2000, 200, 2000), "pipe_sphere": (0, 20, 180)}
    pre, warm, steps = lengths.get(args.workload, (2000, 200, 5000))
    args.precursor = pre if args.precursor is None else args.precursor
    args.warmup = warm if args.warmup is None else args.warmup
    args.steps = steps if args.steps is None else args.steps
    if args.workload == "batch_instances":
        run_batch(args)
        return
    if args.workload == "differentiation_form":
        run_adjoint(args)
        return
    precision = args.precision or default_precision(args.workload)
    w = build_workload(args.workload, precision, args.train, args.junction)
    torch.cuda.set_device(0)
    lat = P.Lattice(w.domain, w.tau, w.u_max, precision)
    if args.precursor > 0 and w.bodies:
        lat.step(args.precursor)
        lat.sync()
    for b in w.bodies:
        lat.add_body(b)
    info = lat.info()
    if args.log_out and w.bodies:
        run_logged(args, lat, w, info, precision)
        return
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
            # MLS points per step: forcing marker and two probes per face, one
            # velocity interpolation per vertex of a soft body
            "markers_per_s": round((info["n_faces"] * 3 + info["n_vertices"]) * args.steps / elapsed, 1)
            if w.bodies else 0,
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
            "peak_copy_measured": measured_copy_gbs(),
            "working_set_in_infinity_cache": bool(bytes_alg < 200e6),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
