"""Writes bifurcation_capsule_oracle.npz: the FP64 oracle's state of the
Y-bifurcation + 2562-vertex capsule workload as the benchmark runs it -- a
particle-free precursor of PRECURSOR steps from rest, then the capsule is
released -- at several step counts after the release (0 = the end of the
precursor), sampled on a fixed seeded set of fluid nodes, plus all vertex
positions.

It also records how far the same trajectory moves when only rounding changes,
from measurement builds of the same oracle source (see oracle.build):
  env_fma_*      the oracle with fused multiply-adds vs the oracle,
  env_reassoc_*  the oracle with reordered sums vs the oracle,
  env_f32_*      the oracle with its populations stored in FP32 vs the oracle,
each as (e_u, e_x) in the measures the parity test uses.  A trajectory that
amplifies rounding (the capsule's motion does, at a rate set by the
workload) cannot be held closer to the oracle than these.

Calls only the oracle and the input generators.

    python tests/golden/make_bifurcation_capsule.py
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

PRECURSOR = 2000
CHECKPOINTS = (0, 50, 200, 1000, 2000, 5200)  # steps after the release
N_SAMPLE = 2048


def run(lib_path, out_path):
    """One trajectory with the oracle library at lib_path (None: the oracle);
    writes the sampled states to out_path."""
    if lib_path:
        oracle.use_library(lib_path)
    w = synth.bifurcation_capsule()
    fluid = np.flatnonzero(w.domain.node_type != synth.SOLID)
    rng = np.random.default_rng(1234)
    sample = np.sort(rng.choice(fluid, N_SAMPLE, replace=False))
    sim = oracle.from_workload(w, with_bodies=False)
    t0 = time.time()
    st = sim.step(PRECURSOR)
    assert st == 0, st
    sim.add_body(w.bodies[0])
    out = {"sample": sample, "checkpoints": np.array(CHECKPOINTS),
           "precursor": np.array(PRECURSOR)}
    done = 0
    for k in CHECKPOINTS:
        st = sim.step(k - done) if k > done else sim.status
        done = k
        rho, u = sim.fields()
        x, _ = sim.body(0)
        out[f"rho_{k}"] = rho[sample]
        out[f"u_{k}"] = u[:, sample]
        out[f"x_{k}"] = x
        out[f"status_{k}"] = np.array(st)
        print(f"  step {k} after release: status {st}, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(out_path, **out)


def errors(a, b, x_release):
    """(e_u, e_x) of state a against state b, as in the parity test."""
    res = {}
    for k in b["checkpoints"]:
        k = int(k)
        uo, xo = b[f"u_{k}"], b[f"x_{k}"]
        e_u = np.abs(a[f"u_{k}"] - uo).max() / np.abs(uo).max()
        disp = np.abs(xo - x_release).max()
        e_x = np.abs(a[f"x_{k}"] - xo).max() / disp if disp > 0 else 0.0
        res[k] = (e_u, e_x)
    return res


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--run":
        run(None if sys.argv[2] == "-" else sys.argv[2], sys.argv[3])
        return
    with tempfile.TemporaryDirectory() as tmp:
        states = {}
        for variant in ("plain", "fma", "reassoc", "store_f32"):
            lib_path = "-"
            if variant != "plain":
                lib_path = oracle.build(variant=variant, path=os.path.join(tmp, f"lib_{variant}.so"))
            out = os.path.join(tmp, f"{variant}.npz")
            print(f"{variant}:", flush=True)
            subprocess.run([sys.executable, os.path.abspath(__file__), "--run", lib_path, out],
                           check=True)
            states[variant] = dict(np.load(out))
    g = states["plain"]
    x_release = synth.bifurcation_capsule().bodies[0].x
    for variant, tag in (("fma", "env_fma"), ("reassoc", "env_reassoc"), ("store_f32", "env_f32")):
        for k, (e_u, e_x) in errors(states[variant], g, x_release).items():
            g[f"{tag}_{k}"] = np.array([e_u, e_x])
            print(f"{tag} step {k}: e_u {e_u:.3e} e_x {e_x:.3e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "bifurcation_capsule_oracle.npz"), **g)


if __name__ == "__main__":
    main()
