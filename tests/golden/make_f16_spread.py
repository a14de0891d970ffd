"""Writes f16_spread.json: how far binary16 population storage alone moves
the small parity cases.  For each case it records (e_u, e_x) of the
oracle's measurement build that rounds the stored populations (their
deviations f - w_i) to binary16 at every step, against the oracle, in the
measures the parity tests use.  An FP16-storage path cannot be held closer
to the oracle than this.

Calls only the oracle and the input generators.

    python tests/golden/make_f16_spread.py
"""
import json
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def cases():
    """name -> (workload, steps, with bodies); the same cases as the FP16
    parity tests."""
    def periodic():
        d = synth.periodic_box(20, 13, 11, body_force=(1e-5, -2e-6, 3e-6))
        rng = np.random.default_rng(1)
        d.init_rho = 1 + 0.01 * rng.standard_normal(d.n_nodes)
        d.init_u = 0.02 * rng.standard_normal(3 * d.n_nodes)
        return synth.Workload("periodic_box", d, [], 0.9, 0.0, "f16s", 7)
    return {
        "periodic_box": (periodic(), 7, False),
        "tiny_pipe": (synth.tiny_pipe(precision="f16s", with_body=False), 40, False),
        "tiny_bifurcation": (synth.tiny_bifurcation(precision="f16s", n_bodies=0), 40, False),
        "pipe_rigid_sphere": (synth.tiny_pipe(precision="f16s", rigid=True), 30, True),
        "pipe_soft_capsule": (synth.tiny_pipe(precision="f16s", rigid=False), 30, True),
        "bifurcation_two_capsules": (synth.tiny_bifurcation(precision="f16s", n_bodies=2), 30, True),
    }


def run(lib_path, out_path):
    if lib_path != "-":
        oracle.use_library(lib_path)
    res = {}
    for name, (w, steps, bodies) in cases().items():
        o = oracle.from_workload(w, with_bodies=bodies, threads=1)
        assert o.step(steps) == 0, name
        _, u = o.fields()
        res[f"{name}_u"] = u
        for i in range(len(w.bodies) if bodies else 0):
            res[f"{name}_x{i}"] = o.body(i)[0]
    np.savez(out_path, **res)


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--run":
        run(sys.argv[2], sys.argv[3])
        return
    with tempfile.TemporaryDirectory() as tmp:
        f16 = oracle.build(variant="store_f16", path=os.path.join(tmp, "f16.so"))
        for lib_path, out in (("-", "plain.npz"), (f16, "f16.npz")):
            subprocess.run([sys.executable, os.path.abspath(__file__), "--run", lib_path,
                            os.path.join(tmp, out)], check=True)
        p = np.load(os.path.join(tmp, "plain.npz"))
        q = np.load(os.path.join(tmp, "f16.npz"))
        out = {}
        for name, (w, steps, bodies) in cases().items():
            fl = w.domain.node_type != synth.SOLID
            up, uq = p[f"{name}_u"], q[f"{name}_u"]
            e_u = np.abs(uq[:, fl] - up[:, fl]).max() / np.abs(up[:, fl]).max()
            e_x = 0.0
            for i, b in enumerate(w.bodies if bodies else []):
                xp, xq = p[f"{name}_x{i}"], q[f"{name}_x{i}"]
                e_x = max(e_x, np.abs(xq - xp).max() / np.abs(xp - b.x).max())
            out[name] = {"steps": steps, "e_u": float(e_u), "e_x": float(e_x)}
            print(f"{name}: e_u {e_u:.3e} e_x {e_x:.3e}", flush=True)
    with open(os.path.join(HERE, "f16_spread.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
