"""Writes adjoint_capsule_fd.npz: central finite differences, taken on the
FP64 oracle, of the differentiation form's objectives with the capsule: the
256x128x40 bifurcation (D = 32, 60 degree semi-aperture) after its
particle-free precursor of PRECURSOR steps from rest, with the 2562-vertex
capsule released and followed for STEPS coupled steps.

Objectives, summed over the steps 1..STEPS after the release:
  J_T  = sum_t D_T(x^t), the capsule's Taylor deformation
         (sqrt(l1) - sqrt(l3)) / (sqrt(l1) + sqrt(l3)) from the largest and
         smallest eigenvalues of the second-moment tensor of its vertices;
  J_up = sum_t sum_{upper outlet nodes} sum_i e_iy f_i^t,
  J_lo = sum_t sum_{lower outlet nodes} sum_i (-e_iy) f_i^t
(the outward fluxes of the two daughters; the flux split is
S = J_up / (J_up + J_lo)).
Parameters (the precursor state held fixed): kappa, the membrane modulus
k_s0 times kappa (the capillary number Ca / kappa), and s, every inlet wall
velocity times s (u_max times s, k_s0 held fixed), each at relative steps
1e-4 and 5e-5.

Stored: the unperturbed (J_T, J_up, J_lo) and, per parameter and step, the
triples at p (1 + h) and p (1 - h).

Calls only the oracle and the input generators.  Nine oracle runs of STEPS
coupled steps, four at a time, after one precursor.

    python tests/golden/make_adjoint_capsule_fd.py
"""
import copy
import multiprocessing
import os
import sys
import tempfile
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

PRECURSOR = 2000
STEPS = 2000
H = (1e-4, 5e-5)


def workload():
    return synth.bifurcation_capsule(precision="f64")


def outlet_nodes(d):
    out = np.flatnonzero(d.node_type == synth.OUTLET)
    y = (out // d.nx) % d.ny
    return out[y == d.ny - 1], out[y == 0]


def taylor(x):
    d = x - x.mean(0)
    lam = np.linalg.eigvalsh(d.T @ d / len(x))
    a, c = np.sqrt(lam[2]), np.sqrt(lam[0])
    return (a - c) / (a + c)


def run(args):
    """(J_T, J_up, J_lo) after the release, with the given scales."""
    kappa, s, pre_path, threads = args
    w = workload()
    w2 = copy.deepcopy(w)
    w2.domain.inlet_u = w.domain.inlet_u * s
    w2.bodies[0].ca = w.bodies[0].ca / kappa
    sim = oracle.from_workload(w2, threads=threads, with_bodies=False)
    sim.set_populations(np.load(pre_path))
    sim.add_body(w2.bodies[0])
    e_y = oracle.lattice()[0][:, 1].astype(np.float64)
    up, lo = outlet_nodes(w.domain)
    jt = ju = jl = 0.0
    for _ in range(STEPS):
        st = sim.step(1)
        assert st == 0, st
        jt += taylor(sim.body(0)[0])
        ju += float(e_y @ sim.populations_at(up).sum(axis=1))
        jl -= float(e_y @ sim.populations_at(lo).sum(axis=1))
    return jt, ju, jl


def main():
    w = workload()
    with tempfile.TemporaryDirectory() as tmp:
        pre = os.path.join(tmp, "pre.npy")
        sim = oracle.from_workload(w, with_bodies=False)
        assert sim.step(PRECURSOR) == 0
        np.save(pre, sim.populations())
        del sim
        jobs = [(1.0, 1.0, pre, 2)]
        for h in H:
            for sg in (1, -1):
                jobs.append((1.0 + sg * h, 1.0, pre, 2))
                jobs.append((1.0, 1.0 + sg * h, pre, 2))
        # fresh interpreters: a child forked after OpenMP ran in this process
        # can hang in the OpenMP runtime
        with ProcessPoolExecutor(4, mp_context=multiprocessing.get_context("spawn")) as ex:
            res = list(ex.map(run, jobs))
    out = {"base": np.array(res[0]), "h": np.array(H), "precursor": np.array(PRECURSOR),
           "steps": np.array(STEPS)}
    k = 1
    for i, h in enumerate(H):
        out[f"kappa_p{i}"], out[f"s_p{i}"] = np.array(res[k]), np.array(res[k + 1])
        out[f"kappa_m{i}"], out[f"s_m{i}"] = np.array(res[k + 2]), np.array(res[k + 3])
        k += 4
    np.savez(os.path.join(HERE, "adjoint_capsule_fd.npz"), **out)
    for key, v in out.items():
        print(key, v)


if __name__ == "__main__":
    main()
