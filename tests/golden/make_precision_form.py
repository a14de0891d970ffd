"""Writes precision_form_oracle.npz: the FP64 oracle's state of the
precision-form workload (bifurcation with a 90 degree semi-aperture on
512x256x64, D = 48, 16 capsules of 2562 vertices) -- a particle-free
precursor of PRECURSOR steps from rest, then the 16 capsules are released --
at several step counts after the release (0 = the end of the precursor),
sampled on a fixed seeded set of fluid nodes and on every VSTRIDE-th vertex
of every capsule.

It also records how far the same trajectory moves when only rounding
changes, from measurement builds of the same oracle source (see
oracle.build), each as (e_u, e_x) against the oracle in the measures the
parity test uses:
  env_fma_*      fused multiply-adds,
  env_reassoc_*  reordered sums,
  env_f32_*      populations stored in FP32,
  env_f16_*      populations (their deviations f - w_i) stored in binary16.
The last one is what FP16 storage alone does to this trajectory.

Calls only the oracle and the input generators.  The five runs go in
parallel; the whole takes about an hour on 8 cores.

    python tests/golden/make_precision_form.py
"""
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

PRECURSOR = 1000
CHECKPOINTS = (0, 100, 500, 2000)  # steps after the release
N_SAMPLE = 4096
VSTRIDE = 8
VARIANTS = (("plain", None), ("fma", "env_fma"), ("reassoc", "env_reassoc"),
            ("store_f32", "env_f32"), ("store_f16", "env_f16"))


def vertex_sample(nv):
    return np.arange(0, nv, VSTRIDE)


def run(lib_path, out_path, threads):
    """One trajectory with the oracle library at lib_path (None: the oracle);
    writes the sampled states to out_path."""
    if lib_path:
        oracle.use_library(lib_path)
    w = synth.precision_form()
    fluid = np.flatnonzero(w.domain.node_type != synth.SOLID)
    rng = np.random.default_rng(1234)
    sample = np.sort(rng.choice(fluid, N_SAMPLE, replace=False))
    sim = oracle.from_workload(w, with_bodies=False, threads=threads)
    t0 = time.time()
    st = sim.step(PRECURSOR)
    assert st == 0, st
    for b in w.bodies:
        sim.add_body(b)
    out = {"sample": sample, "checkpoints": np.array(CHECKPOINTS),
           "precursor": np.array(PRECURSOR), "vstride": np.array(VSTRIDE)}
    done = 0
    for k in CHECKPOINTS:
        st = sim.step(k - done) if k > done else sim.status
        done = k
        rho, u = sim.fields()
        out[f"rho_{k}"] = rho[sample]
        out[f"u_{k}"] = u[:, sample]
        for i, b in enumerate(w.bodies):
            out[f"x_{k}_{i}"] = sim.body(i)[0][vertex_sample(b.nv)]
        out[f"status_{k}"] = np.array(st)
        print(f"  [{os.path.basename(out_path)}] step {k} after release: status {st}, "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(out_path, **out)


def errors(a, b, x_release):
    """(e_u, e_x) of state a against state b, as in the parity test: e_x is
    the largest over the capsules of the position difference relative to
    that capsule's displacement since the release."""
    res = {}
    for k in b["checkpoints"]:
        k = int(k)
        uo = b[f"u_{k}"]
        e_u = np.abs(a[f"u_{k}"] - uo).max() / np.abs(uo).max()
        e_x = 0.0
        for i, x0 in enumerate(x_release):
            xo = b[f"x_{k}_{i}"]
            disp = np.abs(xo - x0).max()
            if disp > 0:
                e_x = max(e_x, np.abs(a[f"x_{k}_{i}"] - xo).max() / disp)
        res[k] = (e_u, e_x)
    return res


def main():
    if len(sys.argv) == 5 and sys.argv[1] == "--run":
        run(None if sys.argv[2] == "-" else sys.argv[2], sys.argv[3], int(sys.argv[4]))
        return
    threads = max(1, (os.cpu_count() or 8) // len(VARIANTS))
    with tempfile.TemporaryDirectory() as tmp:
        procs, outs = [], {}
        for variant, _ in VARIANTS:
            lib_path = "-"
            if variant != "plain":
                lib_path = oracle.build(variant=variant, path=os.path.join(tmp, f"lib_{variant}.so"))
            outs[variant] = os.path.join(tmp, f"{variant}.npz")
            procs.append(subprocess.Popen([sys.executable, os.path.abspath(__file__), "--run",
                                           lib_path, outs[variant], str(threads)]))
        for p in procs:
            if p.wait() != 0:
                raise SystemExit(f"a run failed with status {p.returncode}")
        states = {v: dict(np.load(o)) for v, o in outs.items()}
    g = states["plain"]
    w = synth.precision_form()
    x_release = [b.x[vertex_sample(b.nv)] for b in w.bodies]
    for variant, tag in VARIANTS[1:]:
        for k, (e_u, e_x) in errors(states[variant], g, x_release).items():
            g[f"{tag}_{k}"] = np.array([e_u, e_x])
            print(f"{tag} step {k}: e_u {e_u:.3e} e_x {e_x:.3e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "precision_form_oracle.npz"), **g)


if __name__ == "__main__":
    main()
