"""Writes storage_form.json: which storage form of the populations keeps the
FP64 oracle nearer the exact trajectory.

The particle-free precursor of the Y-bifurcation workload (256 x 128 x 40,
D = 32, Re = 10, tau = 0.7, from rest) runs 2000 steps in four builds of the
same oracle source (see oracle.build):
  ldouble          deviations f - w, fluid state and arithmetic in long double
                   (64-bit significand): the reference, rounding ~2^-64;
  fullpop_ldouble  full populations f, long double: must agree with the
                   reference to long-double rounding (the two forms are the
                   same map in exact arithmetic);
  plain            the oracle: deviations f - w in double;
  fullpop          full populations f in double.
For each, at steps 500, 1000 and 2000, the relative velocity error against
the reference: e_u = max |u - u_ref| / max |u_ref| over all fluid nodes and
over the outlet nodes.

Calls only the oracle and the input generators.

    python tests/golden/make_storage_form.py
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

CHECKPOINTS = (500, 1000, 2000)
BUILDS = ("ldouble", "fullpop_ldouble", "plain", "fullpop")


def run(lib_path, out_path):
    if lib_path:
        oracle.use_library(lib_path)
    w = synth.bifurcation_capsule()
    sim = oracle.from_workload(w, with_bodies=False)
    out, done = {}, 0
    for k in CHECKPOINTS:
        assert sim.step(k - done) == 0
        done = k
        out[f"u{k}"] = sim.fields()[1]
    np.savez(out_path, **out)


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--run":
        run(sys.argv[2] or None, sys.argv[3])
        return
    w = synth.bifurcation_capsule()
    fluid = w.domain.node_type != synth.SOLID
    outlet = w.domain.node_type == 3
    res = {}
    with tempfile.TemporaryDirectory() as tmp:
        for b in BUILDS:
            lib = "" if b == "plain" else oracle.build(variant=b, path=os.path.join(tmp, f"lib_{b}.so"))
            out = os.path.join(tmp, f"{b}.npz")
            print(f"[{b}] 2000 steps", flush=True)
            subprocess.run([sys.executable, __file__, "--run", lib, out], check=True)
            res[b] = dict(np.load(out))
    ref = res["ldouble"]
    table = {}
    for b in BUILDS[1:]:
        table[b] = {}
        for k in CHECKPOINTS:
            u, r = res[b][f"u{k}"], ref[f"u{k}"]
            scale = np.abs(r[:, fluid]).max()
            table[b][str(k)] = {
                "e_u_fluid": float(np.abs(u[:, fluid] - r[:, fluid]).max() / scale),
                "e_u_outlet": float(np.abs(u[:, outlet] - r[:, outlet]).max() / scale),
            }
    doc = {"workload": "Y-bifurcation precursor, 256x128x40, from rest, fluid only",
           "reference": "ldouble (deviations, long double)",
           "checkpoints": list(CHECKPOINTS), "e_u": table}
    with open(os.path.join(HERE, "storage_form.json"), "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc, indent=1))


if __name__ == "__main__":
    main()
