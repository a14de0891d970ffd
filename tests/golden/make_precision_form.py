"""Writes precision_form_oracle.npz: the FP64 oracle's state of the
precision-form workload (bifurcation with a 90 degree semi-aperture on
512x256x64, D = 48, 16 capsules of 2562 vertices) -- a particle-free
precursor of PRECURSOR steps from rest, then the 16 capsules are released --
at several step counts after the release (0 = the end of the precursor):
velocity and density on a fixed seeded set of fluid nodes plus, at each step
count, every NSTRIDE-th fluid node (in index order) within SHELL lattice
spacings of a capsule vertex there (where the capsules' forcing, probes and
vertex velocities act), and every VSTRIDE-th vertex of every capsule.

It also records how far the same trajectory moves when only rounding
changes, from measurement builds of the same oracle source (see
oracle.build), each as (e_u, e_x) against the oracle in the measures the
parity test uses (over all the sampled nodes):
  env_fma_*, env_reassoc_*, env_fma_reassoc_*  fused multiply-adds,
                 reordered sums, both;
  env_f32_*      populations stored in FP32;
  env_float32_*  the fluid state and arithmetic in binary32;
  env_f16_*      populations (their deviations f - w_i) stored in binary16.
The last one is what FP16 storage alone does to this trajectory.

Calls only the oracle and the input generators.  The seven runs go in
parallel, one thread each; the whole takes a few hours on 8 cores.

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
SHELL = 2.7   # a probe 1.2 outside a face plus its support (1.5)
NSTRIDE = 4
VSTRIDE = 2
VARIANTS = (("plain", None), ("fma", "env_fma"), ("reassoc", "env_reassoc"),
            ("fma_reassoc", "env_fma_reassoc"), ("store_f32", "env_f32"), ("float", "env_float32"),
            ("store_f16", "env_f16"))


def vertex_sample(nv):
    return np.arange(0, nv, VSTRIDE)


def run(lib_path, out_path, threads):
    """One trajectory with the oracle library at lib_path (None: the oracle);
    writes the full fields and all positions at the checkpoints to out_path."""
    if lib_path:
        oracle.use_library(lib_path)
    w = synth.precision_form()
    sim = oracle.from_workload(w, with_bodies=False, threads=threads)
    t0 = time.time()
    st = sim.step(PRECURSOR)
    assert st == 0, st
    for b in w.bodies:
        sim.add_body(b)
    out = {}
    done = 0
    for k in CHECKPOINTS:
        st = sim.step(k - done) if k > done else sim.status
        done = k
        rho, u = sim.fields()
        out[f"rho_{k}"], out[f"u_{k}"] = rho, u
        for i in range(len(w.bodies)):
            out[f"x_{k}_{i}"] = sim.body(i)[0]
        out[f"status_{k}"] = np.array(st)
        print(f"  [{os.path.basename(out_path)}] step {k} after release: status {st}, "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez(out_path, **out)


def samples(d, states, nb):
    """The seeded node set, and per checkpoint every NSTRIDE-th fluid node
    within SHELL of a vertex (oracle positions)."""
    from scipy.spatial import cKDTree
    fluid = d.node_type != synth.SOLID
    rng = np.random.default_rng(1234)
    base = np.sort(rng.choice(np.flatnonzero(fluid), N_SAMPLE, replace=False))
    out = {}
    for k in CHECKPOINTS:
        X = np.concatenate([states[f"x_{k}_{i}"] for i in range(nb)])
        lo = np.maximum(np.floor(X.min(0) - SHELL).astype(int), 0)
        hi = np.minimum(np.ceil(X.max(0) + SHELL).astype(int), [d.nx - 1, d.ny - 1, d.nz - 1])
        zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1),
                                 np.arange(lo[0], hi[0] + 1), indexing="ij")
        n = (xx + d.nx * (yy + d.ny * zz)).ravel()
        pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float64)
        dist, _ = cKDTree(X).query(pts, distance_upper_bound=SHELL + 1e-9)
        near = np.sort(n[(dist <= SHELL) & fluid[n]])[::NSTRIDE]
        out[k] = np.union1d(base, near)
    return out


def errors(a, b, sample, x_release, nb):
    """(e_u, e_x) of state a against state b, as in the parity test: e_x is
    the largest over the capsules of the position difference relative to
    that capsule's displacement since the release."""
    res = {}
    for k in CHECKPOINTS:
        uo = b[f"u_{k}"][:, sample[k]]
        e_u = np.abs(a[f"u_{k}"][:, sample[k]] - uo).max() / np.abs(uo).max()
        e_x = 0.0
        for i in range(nb):
            xo = b[f"x_{k}_{i}"][::VSTRIDE]
            disp = np.abs(xo - x_release[i]).max()
            if disp > 0:
                e_x = max(e_x, np.abs(a[f"x_{k}_{i}"][::VSTRIDE] - xo).max() / disp)
        res[k] = (e_u, e_x)
    return res


def main():
    if len(sys.argv) == 5 and sys.argv[1] == "--run":
        run(None if sys.argv[2] == "-" else sys.argv[2], sys.argv[3], int(sys.argv[4]))
        return
    w = synth.precision_form()
    nb = len(w.bodies)
    with tempfile.TemporaryDirectory() as tmp:
        procs, outs = [], {}
        for variant, _ in VARIANTS:
            lib_path = "-"
            if variant != "plain":
                lib_path = oracle.build(variant=variant, path=os.path.join(tmp, f"lib_{variant}.so"))
            outs[variant] = os.path.join(tmp, f"{variant}.npz")
            procs.append(subprocess.Popen([sys.executable, os.path.abspath(__file__), "--run",
                                           lib_path, outs[variant], "1"]))
        for p in procs:
            if p.wait() != 0:
                raise SystemExit(f"a run failed with status {p.returncode}")
        states = {v: dict(np.load(o)) for v, o in outs.items()}
    p = states["plain"]
    sample = samples(w.domain, p, nb)
    g = {"checkpoints": np.array(CHECKPOINTS), "precursor": np.array(PRECURSOR), "vstride": np.array(VSTRIDE),
         "shell": np.array(SHELL), "nstride": np.array(NSTRIDE)}
    for k in CHECKPOINTS:
        g[f"sample_{k}"] = sample[k].astype(np.int32)
        g[f"u_{k}"] = p[f"u_{k}"][:, sample[k]]
        g[f"rho_{k}"] = p[f"rho_{k}"][sample[k]]
        g[f"status_{k}"] = p[f"status_{k}"]
        for i in range(nb):
            g[f"x_{k}_{i}"] = p[f"x_{k}_{i}"][::VSTRIDE]
    x_release = [b.x[::VSTRIDE] for b in w.bodies]
    for variant, tag in VARIANTS[1:]:
        for k, (e_u, e_x) in errors(states[variant], p, sample, x_release, nb).items():
            g[f"{tag}_{k}"] = np.array([e_u, e_x])
            print(f"{tag} step {k}: e_u {e_u:.3e} e_x {e_x:.3e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "precision_form_oracle.npz"), **g)


if __name__ == "__main__":
    main()
