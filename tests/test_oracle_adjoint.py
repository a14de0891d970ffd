"""Pins of the oracle's discrete adjoint (oracle/torch_step.py): the coupled
step written a second time in PyTorch FP64, whose reverse-mode derivative is
the exact derivative of the discrete step.

Its forward trajectory is held to the C oracle's, and its derivatives to
central differences of the C oracle (which shares no code with it), taken at
two step sizes: their gap estimates the difference's own error."""
import copy

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.torch_step import TorchSim, taylor_deformation

W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None]
EX = np.array([0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0])


def _cases():
    return {"pipe_soft": synth.tiny_pipe(precision="f64", rigid=False),
            "bifurcation": synth.tiny_bifurcation(precision="f64", n_bodies=1)}


@pytest.mark.parametrize("name", ["pipe_soft", "bifurcation"])
def test_torch_step_follows_the_oracle(name):
    w = _cases()[name]
    ts = TorchSim(w)
    st, prm = ts.initial_state(), ts.params()
    with torch.no_grad():
        for _ in range(12):
            st, rho, u = ts.step(st, prm)
    o = oracle.from_workload(w)
    assert o.step(12) == 0
    fl = w.domain.node_type != synth.SOLID
    _, uo = o.fields()
    assert np.abs(u.numpy()[:, fl] - uo[:, fl]).max() < 1e-12 * np.abs(uo[:, fl]).max()
    assert np.abs((st["g"].numpy() + W19)[:, fl] - o.populations()[:, fl]).max() < 1e-15
    assert np.abs(st["bodies"][0][0].numpy() - o.body(0)[0]).max() < 1e-13
    # velocities are differences of positions near 10-20 lu: rounding ~1e-14
    assert np.abs(st["bodies"][0][2].numpy() - o.body(0)[1]).max() < 1e-13


def _objective(w, n, seed=3, theta=3.0):
    """J = <lam, g^n> + sum_t <w, g^t> + theta sum_t D_T(x^t): a seeded
    terminal weight, the x-momentum flux of one cross-section, and the
    capsule's Taylor deformation after every step."""
    rng = np.random.default_rng(seed)
    N = w.domain.n_nodes
    fl = w.domain.node_type != synth.SOLID
    lam = rng.normal(size=(19, N)) * fl
    x = np.arange(N) % w.domain.nx
    wobs = np.zeros((19, N))
    wobs[:, (x == w.domain.nx - 3) & fl] = EX[:, None]
    return lam, wobs, theta


def _J_torch(w, n, lam, wobs, theta):
    ts = TorchSim(w)
    st, prm = ts.initial_state(), ts.params()
    for k in ("s", "kappa", "tau"):
        prm[k].requires_grad_(True)
    J = 0.0
    for _ in range(n):
        st, _, _ = ts.step(st, prm)
        J = J + (torch.tensor(wobs) * st["g"]).sum() + theta * taylor_deformation(st["bodies"][0][0])
    J = J + (torch.tensor(lam) * st["g"]).sum()
    J.backward()
    return J.item(), {k: prm[k].grad.item() for k in ("s", "kappa", "tau")}


def _J_oracle(w, n, lam, wobs, theta, s=1.0, kappa=1.0, tau=None):
    """The C oracle's J with the inlet velocities times s, the membrane
    modulus k_s0 times kappa and the relaxation time tau (k_s0 held fixed:
    the capillary number follows nu)."""
    tau = w.tau if tau is None else tau
    w2 = copy.deepcopy(w)
    w2.domain.inlet_u = w.domain.inlet_u * s
    for b in w2.bodies:
        b.ca = b.ca / kappa * ((tau - 0.5) / (w.tau - 0.5))
    w2.tau = tau
    o = oracle.from_workload(w2)
    J = 0.0
    for _ in range(n):
        assert o.step(1) == 0
        J += (wobs * (o.populations() - W19)).sum()
        J += theta * float(taylor_deformation(torch.tensor(o.body(0)[0])))
    return J + (lam * (o.populations() - W19)).sum()


@pytest.mark.parametrize("name", ["pipe_soft", "bifurcation"])
def test_torch_adjoint_matches_oracle_differences(name):
    """dJ/ds (inlet velocity), dJ/dkappa (membrane stiffness) and dJ/dtau
    from reverse-mode differentiation of the torch step, against central
    differences of the C oracle at h and h/2 (relative step 1e-4)."""
    w = _cases()[name]
    n = 10
    lam, wobs, theta = _objective(w, n)
    J, grad = _J_torch(w, n, lam, wobs, theta)
    assert abs(J - _J_oracle(w, n, lam, wobs, theta)) < 1e-12 * abs(J)
    for k in ("s", "kappa", "tau"):
        base = w.tau if k == "tau" else 1.0
        fd = []
        for h in (1e-4, 5e-5):
            jp = _J_oracle(w, n, lam, wobs, theta, **{k: base * (1 + h)})
            jm = _J_oracle(w, n, lam, wobs, theta, **{k: base * (1 - h)})
            fd.append((jp - jm) / (2 * h * base))
        gap = abs(fd[0] - fd[1])
        assert abs(grad[k] - fd[1]) <= 1e-8 * abs(grad[k]) + 4 * gap, (k, grad[k], fd)


def test_taylor_deformation_of_a_stretched_sphere():
    """The vertex second-moment tensor of an icosphere is isotropic (its
    icosahedral symmetry admits no other symmetric tensor), so stretching it
    by (a, b, c) along rotated axes makes the eigenvalues proportional to
    a^2, b^2, c^2 and D_T = (a - c) / (a + c) exactly (the Taylor deformation
    of the stretched sphere).  Picking the middle eigenvalue, dropping the
    square roots or not centring the vertices fails this."""
    from scipy.spatial.transform import Rotation

    X, _ = synth.icosphere(3, 1.0, (0.0, 0.0, 0.0), tilt=True)
    d = X - X.mean(0)
    M = d.T @ d / len(X)
    assert np.abs(M - np.eye(3) * M.trace() / 3).max() < 1e-14
    Q = Rotation.from_rotvec([0.4, -1.1, 0.7]).as_matrix()
    for abc in [(1.3, 1.0, 0.8), (2.0, 0.5, 0.5), (0.7, 1.6, 1.1), (1.0, 1.0, 1.0)]:
        s = np.array(abc)
        Y = ((X @ Q) * s) @ Q.T + np.array([10.0, -3.0, 7.5])
        D = float(taylor_deformation(torch.tensor(Y)))
        want = (s.max() - s.min()) / (s.max() + s.min())
        assert abs(D - want) < 1e-12, (abc, D, want)
