"""Writes bifurcation_capsule_oracle.npz: the FP64 oracle's state of the
Y-bifurcation + 2562-vertex capsule workload as the benchmark runs it -- a
particle-free precursor of PRECURSOR steps from rest, then the capsule is
released -- at several step counts after the release (0 = the end of the
precursor): the velocity and density on a fixed seeded set of fluid nodes,
plus, at each step count, on every fluid node within NEAR lattice spacings of
the capsule's bounding box there (the region its forcing, probes and vertex
velocities reach), and all vertex positions.

It also records how far the same trajectory moves when only rounding changes,
from measurement builds of the same oracle source (see oracle.build): for
FP64, fused multiply-adds, reordered sums and both; for FP32, the populations
stored in FP32, and the fluid state and arithmetic in FP32.  Each is stored
as (e_u, e_x) against the oracle in the measures the parity test uses (over
all the sampled nodes), under env_<build>_<step>.  A trajectory that
amplifies rounding (the capsule's motion does) cannot be held closer to the
oracle than these realizations scatter.

Calls only the oracle and the input generators.  Six runs of 7200 steps.

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
NEAR = 3.0
BUILDS = {"fma": "env_fma", "reassoc": "env_reassoc", "fma_reassoc": "env_fma_reassoc",
          "store_f32": "env_f32", "float": "env_float32"}


def run(lib_path, out_path):
    """One trajectory with the oracle library at lib_path (None: the oracle);
    writes the full velocity and density fields and the positions at the
    checkpoints to out_path."""
    if lib_path:
        oracle.use_library(lib_path)
    w = synth.bifurcation_capsule()
    sim = oracle.from_workload(w, with_bodies=False)
    t0 = time.time()
    st = sim.step(PRECURSOR)
    assert st == 0, st
    sim.add_body(w.bodies[0])
    out = {}
    done = 0
    for k in CHECKPOINTS:
        st = sim.step(k - done) if k > done else sim.status
        done = k
        rho, u = sim.fields()
        out[f"rho_{k}"], out[f"u_{k}"], out[f"x_{k}"] = rho, u, sim.body(0)[0]
        out[f"status_{k}"] = np.array(st)
        print(f"  step {k} after release: status {st}, {time.time() - t0:.0f} s", flush=True)
    np.savez(out_path, **out)


def samples(d, states):
    """The seeded node set, and per checkpoint the fluid nodes within NEAR of
    the capsule's bounding box (oracle positions)."""
    fluid = d.node_type != synth.SOLID
    rng = np.random.default_rng(1234)
    base = np.sort(rng.choice(np.flatnonzero(fluid), N_SAMPLE, replace=False))
    n = np.arange(d.n_nodes)
    x, y, z = n % d.nx, (n // d.nx) % d.ny, n // (d.nx * d.ny)
    out = {}
    for k in CHECKPOINTS:
        X = states[f"x_{k}"]
        lo, hi = X.min(0) - NEAR, X.max(0) + NEAR
        near = fluid & (x >= lo[0]) & (x <= hi[0]) & (y >= lo[1]) & (y <= hi[1]) & (z >= lo[2]) & (z <= hi[2])
        out[k] = np.union1d(base, np.flatnonzero(near))
    return out


def errors(a, b, sample, x_release):
    """(e_u, e_x) of state a against state b, as in the parity test."""
    res = {}
    for k in CHECKPOINTS:
        uo, xo = b[f"u_{k}"][:, sample[k]], b[f"x_{k}"]
        e_u = np.abs(a[f"u_{k}"][:, sample[k]] - uo).max() / np.abs(uo).max()
        disp = np.abs(xo - x_release).max()
        e_x = np.abs(a[f"x_{k}"] - xo).max() / disp if disp > 0 else 0.0
        res[k] = (e_u, e_x)
    return res


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--run":
        run(None if sys.argv[2] == "-" else sys.argv[2], sys.argv[3])
        return
    w = synth.bifurcation_capsule()
    with tempfile.TemporaryDirectory() as tmp:
        states = {}
        for variant in ("plain", *BUILDS):
            lib_path = "-"
            if variant != "plain":
                lib_path = oracle.build(variant=variant, path=os.path.join(tmp, f"lib_{variant}.so"))
            out = os.path.join(tmp, f"{variant}.npz")
            print(f"{variant}:", flush=True)
            subprocess.run([sys.executable, os.path.abspath(__file__), "--run", lib_path, out], check=True)
            states[variant] = dict(np.load(out))
    p = states["plain"]
    sample = samples(w.domain, p)
    g = {"checkpoints": np.array(CHECKPOINTS), "precursor": np.array(PRECURSOR), "near": np.array(NEAR)}
    for k in CHECKPOINTS:
        g[f"sample_{k}"] = sample[k]
        g[f"u_{k}"] = p[f"u_{k}"][:, sample[k]]
        g[f"rho_{k}"] = p[f"rho_{k}"][sample[k]]
        g[f"x_{k}"] = p[f"x_{k}"]
        g[f"status_{k}"] = p[f"status_{k}"]
    x_release = w.bodies[0].x
    for variant, tag in BUILDS.items():
        for k, (e_u, e_x) in errors(states[variant], p, sample, x_release).items():
            g[f"{tag}_{k}"] = np.array([e_u, e_x])
            print(f"{tag} step {k}: e_u {e_u:.3e} e_x {e_x:.3e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "bifurcation_capsule_oracle.npz"), **g)


if __name__ == "__main__":
    main()
