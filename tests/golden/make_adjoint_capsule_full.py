"""Writes adjoint_capsule_full.npz: the oracle's discrete adjoint of the
differentiation form's coupled objective at full size, for a horizon the
CPU can differentiate.

Set-up: the 256x128x40 bifurcation (D = 32, 60 degree semi-aperture), FP64,
after its particle-free precursor of PRECURSOR steps from rest (C oracle),
with the 2562-vertex capsule released and followed for STEPS coupled steps
(oracle/torch_step.py, whose forward is pinned to the C oracle).

Objective: J = <lam, g^n> + sum_{t=1..n} <w_up, g^t> + THETA sum_{t=1..n} D_T(x^t)
with lam = synth.terminal_weights(domain, SEED), w_up the upper daughter's
outward flux (synth.outlet_flux_weights) and D_T the capsule's Taylor
deformation.

The reverse sweep is checkpointed by hand: the state is kept every SEG
steps; each segment is recomputed without gradients, then its steps are
taken in reverse, each one differentiated by torch reverse mode (the
vector-Jacobian product of one step, accumulated into the parameter
gradients).

Stored: J's two parts, the parameter gradients (inlet scale s, body force F,
tau, stiffness scale kappa), dJ/d(x^0, x^{-1}, u_v^0) of the capsule, and
dJ/dg^0 at SAMPLES seeded flat indices of [19, N] with its 2-norm.

Calls only the oracle and the input generators.

    python tests/golden/make_adjoint_capsule_full.py
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle.torch_step import WGT, TorchSim, taylor_deformation  # noqa: E402

PRECURSOR = 2000
STEPS = 200
SEG = 20
THETA = 1.0
SEED = 11
SAMPLES = 4096


def workload():
    return synth.bifurcation_capsule(precision="f64")


def _say(msg):
    print(time.strftime("%H:%M:%S"), msg, flush=True)


def _detach(st):
    return {"g": st["g"].detach(), "bodies": [tuple(t.detach() for t in b) for b in st["bodies"]]}


def _leaf(st):
    return {"g": st["g"].detach().clone().requires_grad_(True),
            "bodies": [tuple(t.detach().clone().requires_grad_(True) for t in b) for b in st["bodies"]]}


def main():
    torch.set_num_threads(8)
    w = workload()
    d = w.domain
    sim = oracle.from_workload(w, with_bodies=False)
    assert sim.step(PRECURSOR) == 0
    f = sim.populations()
    del sim
    _say("precursor done")
    ts = TorchSim(w)
    openm = torch.tensor(ts.open, dtype=torch.float64)
    st0 = ts.initial_state()
    st0["g"] = (torch.from_numpy(f) - torch.tensor(WGT)[:, None]) * openm
    prm = ts.params()
    lam = torch.from_numpy(synth.terminal_weights(d, SEED))
    w_up = torch.from_numpy(synth.outlet_flux_weights(d)[0])

    starts = []
    st = st0
    Jw, Jt = 0.0, 0.0
    with torch.no_grad():
        for t in range(STEPS):
            if t % SEG == 0:
                starts.append(st)
            st, _, _ = ts.step(st, prm)
            Jw += float((w_up * st["g"]).sum())
            Jt += float(taylor_deformation(st["bodies"][0][0]))
        Jw += float((lam * st["g"]).sum())
    _say(f"forward done J = {Jw!r}, {Jt!r}")

    for k in ("s", "kappa", "tau", "F"):
        prm[k].requires_grad_(True)
    pgrad = {k: torch.zeros_like(v) for k, v in prm.items()}
    P, Q, V = st["bodies"][0]
    with torch.enable_grad():
        Pl = P.detach().clone().requires_grad_(True)
        (dP,) = torch.autograd.grad(THETA * taylor_deformation(Pl), Pl)
    adj = {"g": lam + w_up, "bodies": [(dP, torch.zeros_like(Q), torch.zeros_like(V))]}
    for si in range(len(starts) - 1, -1, -1):
        t0 = si * SEG
        states = [starts[si]]
        with torch.no_grad():
            for t in range(t0, min(t0 + SEG, STEPS) - 1):
                states.append(ts.step(states[-1], prm)[0])
        for t in range(min(t0 + SEG, STEPS) - 1, t0 - 1, -1):
            x = _leaf(states[t - t0])
            with torch.enable_grad():
                y, _, _ = ts.step(x, prm)
                (Py, Qy, Vy), (aP, aQ, aV) = y["bodies"][0], adj["bodies"][0]
                L = (adj["g"] * y["g"]).sum() + (aP * Py).sum() + (aQ * Qy).sum() + (aV * Vy).sum()
                if t >= 1:  # the terms of J at the step's input state
                    L = L + (w_up * x["g"]).sum() + THETA * taylor_deformation(x["bodies"][0][0])
                leaves = [x["g"], *x["bodies"][0], prm["s"], prm["kappa"], prm["tau"], prm["F"]]
                gr = torch.autograd.grad(L, leaves, allow_unused=True)
            z = [torch.zeros_like(v) if gv is None else gv for gv, v in zip(gr, leaves)]
            adj = {"g": z[0], "bodies": [(z[1], z[2], z[3])]}
            for k, gv in zip(("s", "kappa", "tau", "F"), z[4:]):
                pgrad[k] += gv
            del x, y, L, gr
        _say(f"segment {si} done")
    g0 = adj["g"].numpy()
    rng = np.random.default_rng(SEED + 1)
    fl = np.flatnonzero(np.tile(d.node_type != synth.SOLID, 19))
    idx = np.sort(rng.choice(fl, SAMPLES, replace=False))
    out = {"J": np.array([Jw, Jt]),
           "grad": np.array([float(pgrad["s"]), *pgrad["F"].numpy(), float(pgrad["tau"]), float(pgrad["kappa"])]),
           "body": np.stack([t.numpy() for t in adj["bodies"][0]]),
           "g0_idx": idx, "g0_val": g0.reshape(-1)[idx], "g0_norm": np.array(np.linalg.norm(g0)),
           "g0_max": np.array(np.abs(g0).max()),
           "precursor": np.array(PRECURSOR), "steps": np.array(STEPS), "theta": np.array(THETA),
           "seed": np.array(SEED)}
    np.savez_compressed(os.path.join(HERE, "adjoint_capsule_full.npz"), **out)
    for k in ("J", "grad", "g0_norm", "g0_max"):
        print(k, out[k])


if __name__ == "__main__":
    main()
