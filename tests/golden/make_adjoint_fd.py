"""Writes adjoint_fd.npz: central finite differences, taken on the FP64
oracle, of two time-integrated observables of the differentiation-form
workload -- the 256x128x40 bifurcation of D = 32 (60 degree
semi-aperture) from rest, fluid only, over STEPS steps -- with respect to
the inlet-velocity scale s (every inlet wall velocity times s) and the
uniform body force F.

Observables (outward volume fluxes through the two daughter outlets, on the
faces y = ny - 1 and y = 0, summed over steps 1..STEPS):
  J_up = sum_t sum_{upper outlet nodes} sum_i e_iy f_i^t
  J_lo = sum_t sum_{lower outlet nodes} sum_i (-e_iy) f_i^t
The flux split is S = J_up / (J_up + J_lo).

Stored: the unperturbed J_up, J_lo, and for each parameter p and step h in
H[p] the pairs (J_up, J_lo) at p + h and p - h.  The adjoint test forms the
differences itself.

Calls only the oracle and the input generators.  Eleven oracle runs, four
at a time; about ten minutes on 8 cores.

    python tests/golden/make_adjoint_fd.py
"""
import copy
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

STEPS = 2000
# s is relative (1e-4, as the differentiation form asks); F is absolute,
# 1e-4 of the force that would drive the inlet's Poiseuille flow
# (8 nu u_max / R^2 ~ 4e-6 at this size)
H = {"s": (1e-4, 5e-5), "Fx": (4e-10,), "Fy": (4e-10, 2e-10)}


def workload():
    """The differentiation-form workload: the bifurcation of the single
    capsule case, without its capsule, in FP64."""
    return synth.bifurcation_capsule(precision="f64")


def outlet_nodes(d):
    """(upper, lower) daughter outlet node indices."""
    out = np.flatnonzero(d.node_type == synth.OUTLET)
    y = (out // d.nx) % d.ny
    return out[y == d.ny - 1], out[y == 0]


def weights(d):
    """[19][N] weights of the per-step fluxes J_up and J_lo (the w of the
    objective sum_t <w, f^t>)."""
    e = oracle.lattice()[0]
    up, lo = outlet_nodes(d)
    w_up = np.zeros((19, d.n_nodes))
    w_lo = np.zeros((19, d.n_nodes))
    w_up[:, up] = e[:, 1][:, None]
    w_lo[:, lo] = -e[:, 1][:, None]
    return w_up, w_lo


def fluxes(d, tau, u_max, steps, threads=2):
    """(J_up, J_lo) of the oracle's trajectory on domain d."""
    e_y = oracle.lattice()[0][:, 1].astype(np.float64)
    up, lo = outlet_nodes(d)
    sim = oracle.OracleSim(d, tau, u_max, threads=threads)
    j_up = j_lo = 0.0
    for _ in range(steps):
        st = sim.step(1)
        assert st == 0, st
        j_up += float(e_y @ sim.populations_at(up).sum(axis=1))
        j_lo -= float(e_y @ sim.populations_at(lo).sum(axis=1))
    return j_up, j_lo


def perturbed(d, p, h):
    q = copy.copy(d)
    if p == "s":
        q.inlet_u = d.inlet_u * (1.0 + h)
    else:
        f = list(d.body_force)
        f["xyz".index(p[1])] += h
        q.body_force = tuple(f)
    return q


def _run(job):
    p, h = job
    w = workload()
    d = w.domain if p is None else perturbed(w.domain, p, h)
    r = fluxes(d, w.tau, w.u_max, STEPS)
    print(f"  {p} {h:+.1e}: J_up {r[0]:.15e} J_lo {r[1]:.15e}" if p else
          f"  base: J_up {r[0]:.15e} J_lo {r[1]:.15e}", flush=True)
    return r


def main():
    jobs = [(None, 0.0)] + [(p, sg * h) for p, hs in H.items() for h in hs for sg in (1, -1)]
    with ProcessPoolExecutor(4) as ex:
        res = dict(zip(jobs, ex.map(_run, jobs)))
    out = {"steps": np.array(STEPS), "base": np.array(res[(None, 0.0)])}
    for p, hs in H.items():
        out[f"h_{p}"] = np.array(hs)
        out[f"plus_{p}"] = np.array([res[(p, h)] for h in hs])
        out[f"minus_{p}"] = np.array([res[(p, -h)] for h in hs])
    np.savez(os.path.join(HERE, "adjoint_fd.npz"), **out)


if __name__ == "__main__":
    main()
