"""Writes facing_pair_spread.json: how far the facing-pair parity case (two
icospheres of 162 vertices, one centroid pair half a spacing apart, fluid
at rest, 20 steps) moves when only rounding changes.  For the soft and the
rigid pair it records (e_u, e_x) of the oracle's measurement builds with
fused multiply-adds ("fma") and with reordered sums ("reassoc") against the
oracle, in the measures the parity test uses.  The soft pair stirs the fluid
only weakly (max |u| ~ 3e-4) while its stiff membrane amplifies rounding, so
its relative velocity error cannot be held below a few 1e-12.

Calls only the oracle and the input generators.

    python tests/golden/make_facing_pair.py
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

STEPS = 20


def workload(rigid):
    return synth.facing_pair(0.5, subdiv=2, rigid=rigid, fixed=False)


def run(lib_path, rigid, out_path):
    if lib_path != "-":
        oracle.use_library(lib_path)
    w = workload(rigid)
    o = oracle.from_workload(w, threads=1)
    assert o.step(STEPS) == 0
    _, u = o.fields()
    np.savez(out_path, u=u, **{f"x{i}": o.body(i)[0] for i in range(len(w.bodies))})


def main():
    if len(sys.argv) == 5 and sys.argv[1] == "--run":
        run(sys.argv[2], sys.argv[3] == "1", sys.argv[4])
        return
    res = {}
    with tempfile.TemporaryDirectory() as tmp:
        for rigid in (False, True):
            w = workload(rigid)
            fl = w.domain.node_type != synth.SOLID
            states = {}
            for variant in ("plain", "fma", "reassoc"):
                lib_path = "-"
                if variant != "plain":
                    lib_path = oracle.build(variant=variant, path=os.path.join(tmp, f"{variant}.so"))
                out = os.path.join(tmp, f"{variant}_{int(rigid)}.npz")
                subprocess.run([sys.executable, os.path.abspath(__file__), "--run", lib_path,
                                str(int(rigid)), out], check=True)
                states[variant] = np.load(out)
            p = states["plain"]
            for variant in ("fma", "reassoc"):
                q = states[variant]
                e_u = np.abs(q["u"][:, fl] - p["u"][:, fl]).max() / np.abs(p["u"][:, fl]).max()
                e_x = max(np.abs(q[f"x{i}"] - p[f"x{i}"]).max() / np.abs(p[f"x{i}"] - b.x).max()
                          for i, b in enumerate(w.bodies))
                res[f"{'rigid' if rigid else 'soft'}_{variant}"] = [float(e_u), float(e_x)]
                print(f"rigid={rigid} {variant}: e_u {e_u:.3e} e_x {e_x:.3e}", flush=True)
    with open(os.path.join(HERE, "facing_pair_spread.json"), "w") as f:
        json.dump({"steps": STEPS, "spread": res}, f, indent=1)


if __name__ == "__main__":
    main()
