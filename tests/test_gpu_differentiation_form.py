"""The differentiation form at full size: the 256x128x40 bifurcation (D = 32,
60 degree semi-aperture) after its particle-free precursor of 2000 steps,
with the 2562-vertex capsule released; the coupled adjoint (lbm_adjoint_run,
FP64 adjoint, checkpoints every 100 steps) against

* the oracle's central differences over 2000 coupled steps, with the FP32
  forward (tests/golden/make_adjoint_capsule_fd.py): the capsule's summed
  Taylor deformation J_T and the daughters' outward fluxes J_up, J_lo, in
  the inlet-velocity scale s and the membrane-stiffness scale kappa;
* the oracle's discrete adjoint (reverse-mode differentiation of the coupled
  step in PyTorch FP64) over 200 coupled steps, FP64 and FP32 forward
  (tests/golden/make_adjoint_capsule_full.py).

Central differences of this objective are noisy: the MLS support of a point
is the 3x3x3 block around its nearest node, so the discrete trajectory jumps
wherever a marker crosses a half-integer plane, and the truncated weight of
the node that leaves the block is not small (exp(-(1.5/0.78)^2) ~ 0.025).
The adjoint is the derivative within one smooth piece; differences at
h = 1e-4 (relative) take in many such jumps.  The bar for each derivative is
therefore the differences' own spread: the gap between the estimates at
h = 1e-4 and 5e-5, plus 2 % of the estimate.  For J_T in s the two
estimates disagree by more than their size (the bar is loose there); the
exact derivative at full size is checked against the oracle's adjoint."""
import os
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PRECURSOR = 2000
K = 100


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2207_06043_amd as P
    P.load_library()
    return P


def _released(P, precision):
    w = synth.bifurcation_capsule(precision="f64")
    lat = P.Lattice(w.domain, w.tau, w.u_max, precision)
    lat.step(PRECURSOR)
    lat.sync()
    lat.add_body(w.bodies[0])
    return w, lat


def _fd(g, p, i, k):
    h = float(g["h"][i])
    return (g[f"{p}_p{i}"][k] - g[f"{p}_m{i}"][k]) / (2.0 * h)


def test_gradients_match_the_oracle_central_differences(lib):
    g = np.load(os.path.join(GOLD, "adjoint_capsule_fd.npz"))
    steps = int(g["steps"])
    assert int(g["precursor"]) == PRECURSOR
    _say(f"[differentiation] fp32 forward, {steps} steps, K = {K}")
    w, lat = _released(lib, "f32")
    w_up, w_lo = (torch.from_numpy(a) for a in synth.outlet_flux_weights(w.domain))
    _, gT, _, JT = lat.adjoint_run(steps, None, None, taylor_weight=1.0, checkpoint_every=K)
    _, gU, _, JU = lat.adjoint_run(steps, None, w_up, checkpoint_every=K)
    _, gL, _, JL = lat.adjoint_run(steps, None, w_lo, checkpoint_every=K)
    J = np.array([JT[1], JU[0], JL[0]])
    _say(f"[differentiation] J = {J}, oracle {g['base']}")
    # the FP32 forward against the FP64 oracle over 4000 steps
    assert np.all(np.abs(J - g["base"]) <= 1e-4 * np.abs(g["base"]))
    adj = {"s": [float(gT[0]), float(gU[0]), float(gL[0])],
           "kappa": [float(gT[5]), float(gU[5]), float(gL[5])]}
    for p in ("s", "kappa"):
        for k, name in enumerate(("J_T", "J_up", "J_lo")):
            d1, d2 = _fd(g, p, 0, k), _fd(g, p, 1, k)
            bar = abs(d1 - d2) + 0.02 * abs(d1)
            _say(f"  d{name}/d{p}: adjoint {adj[p][k]:.6g}  FD(1e-4) {d1:.6g}  FD(5e-5) {d2:.6g}  bar {bar:.3g}")
            assert abs(adj[p][k] - d1) <= bar, (name, p)
    # the flux split S = J_up / (J_up + J_lo) and its derivatives
    Ju, Jl = J[1], J[2]
    for p in ("s", "kappa"):
        dS = (adj[p][1] * Jl - Ju * adj[p][2]) / (Ju + Jl) ** 2
        gb = g["base"]
        fd = []
        for i in (0, 1):
            pp, mm = g[f"{p}_p{i}"], g[f"{p}_m{i}"]
            fd.append((pp[1] / (pp[1] + pp[2]) - mm[1] / (mm[1] + mm[2])) / (2 * float(g["h"][i])))
        _say(f"  dS/d{p}: adjoint {dS:.6g}  FD {fd[0]:.6g} {fd[1]:.6g}  (S = {gb[1] / (gb[1] + gb[2]):.8f})")
        assert abs(dS - fd[0]) <= abs(fd[0] - fd[1]) + 0.02 * abs(fd[0]) + 1e-9


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gradients_match_the_oracle_adjoint(lib, precision):
    ref = np.load(os.path.join(GOLD, "adjoint_capsule_full.npz"))
    steps, theta, seed = int(ref["steps"]), float(ref["theta"]), int(ref["seed"])
    assert int(ref["precursor"]) == PRECURSOR
    _say(f"[differentiation] oracle adjoint, {precision} forward, {steps} steps, K = {K}")
    w, lat = _released(lib, precision)
    lam = torch.from_numpy(synth.terminal_weights(w.domain, seed))
    w_up = torch.from_numpy(synth.outlet_flux_weights(w.domain)[0])
    g0, grad, bg, J = lat.adjoint_run(steps, lam, w_up, taylor_weight=theta, taylor_body=0,
                                      checkpoint_every=K, body_grad=True)
    g0 = g0.cpu().numpy().reshape(-1)
    grad, bg, J = grad.cpu().numpy(), bg.cpu().numpy(), np.array(J)
    eJ = np.abs(J - ref["J"]) / np.abs(ref["J"])
    eg = np.abs(grad - ref["grad"]) / np.abs(ref["grad"])
    eb = np.abs(bg - ref["body"]).max() / np.abs(ref["body"]).max()
    e0 = np.abs(g0[ref["g0_idx"]] - ref["g0_val"]).max() / float(ref["g0_max"])
    en = abs(np.linalg.norm(g0) - float(ref["g0_norm"])) / float(ref["g0_norm"])
    _say(f"  J {J} rel {eJ}\n  grad rel {eg}\n  body {eb:.3g} g0 {e0:.3g} |g0| {en:.3g}")
    # FP64: the precursor states agree to rounding (~1e-13 after 2000
    # steps), and the derivatives follow them smoothly over the horizon
    # (measured up to 2.6e-13); FP32: the forward states carry FP32 rounding
    # into every Jacobian (measured up to 1.7e-6).
    tol = 1e-11 if precision == "f64" else 1e-5
    assert eJ.max() < tol
    assert eg.max() < tol and eb < tol and e0 < tol and en < tol
