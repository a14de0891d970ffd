"""The paper's campaign configurations on the GPU, against the oracle:
trains of three capsules (all soft, one rigid sphere in the middle, three
rigid spheres) in a bifurcation with the smooth (trapezoidal) junction, the
sharp-junction counterpart, and the logged relative surface strain dS(t)
with the damage stop."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2207_06043_amd as P
    P.load_library()
    return P


def _errors(lat, orc, w):
    fl = w.domain.node_type != synth.SOLID
    _, ug = lat.fields()
    ug = ug.cpu().numpy()
    _, uo = orc.fields()
    e_u = np.abs(ug[:, fl] - uo[:, fl]).max() / np.abs(uo[:, fl]).max()
    ex = []
    for b in range(len(w.bodies)):
        xo = orc.body(b)[0]
        disp = np.abs(xo - w.bodies[b].x).max()
        ex.append(np.abs(lat.body(b)[0].cpu().numpy() - xo).max() / disp)
    return e_u, max(ex)


def _released(lib, w, precursor, steps):
    """GPU and oracle: a particle-free precursor, then the bodies released
    and `steps` coupled steps (the capsules move a good part of a lattice
    spacing, so the displacement-normalised e_x is well conditioned)."""
    lat = lib.from_workload(w, with_bodies=False)
    lat.step(precursor)
    for b in w.bodies:
        lat.add_body(b)
    lat.step(steps)
    assert lat.sync(raise_on_stop=False) == 0
    orc = oracle.from_workload(w, with_bodies=False)
    assert orc.step(precursor) == 0
    for b in w.bodies:
        orc.add_body(b)
    assert orc.step(steps) == 0
    return lat, orc


@pytest.mark.parametrize("train", ["soft", "rigid_middle", "all_rigid"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_capsule_train_matches_oracle(lib, train, precision):
    w = synth.tiny_train(train, precision=precision)
    _say(f"[campaign] train {train} {precision}: 300-step precursor, 30 steps")
    lat, orc = _released(lib, w, 300, 30)
    e_u, e_x = _errors(lat, orc, w)
    _say(f"    e_u {e_u:.2e}  e_x {e_x:.2e}")
    assert e_u <= TOL[precision] and e_x <= TOL[precision]


@pytest.mark.parametrize("junction", ["sharp", "smooth"])
def test_junctions_match_oracle(lib, junction):
    w = synth.tiny_train("soft", junction=junction)
    w.bodies = []
    _say(f"[campaign] {junction} junction, fluid only, 60 steps")
    lat = lib.from_workload(w)
    lat.step(60)
    orc = oracle.from_workload(w)
    assert orc.step(60) == 0
    fl = w.domain.node_type != synth.SOLID
    _, ug = lat.fields()
    _, uo = orc.fields()
    e_u = np.abs(ug.cpu().numpy()[:, fl] - uo[:, fl]).max() / np.abs(uo[:, fl]).max()
    assert e_u <= 1e-12


def test_logged_surface_strain_matches_oracle(lib):
    """campaign.log_run: dS = S/S0 - 1 of every capsule every 10 steps, equal
    to the oracle's surfaces at the same steps."""
    w = synth.tiny_train("soft")
    _say("[campaign] logged dS(t)")
    lat, orc = _released(lib, w, 300, 0)
    log = lib.campaign.log_run(lat, 30, 10, w.u_max, 12.0)
    assert log["status"] == "ok" and log["step"] == [0, 10, 20, 30]
    S0 = [orc.body_diag(b)["S0"] for b in range(3)]
    for k, st in enumerate(log["step"]):
        if st:
            assert orc.step(10) == 0
        for b in range(3):
            dS = orc.body_diag(b)["S"] / S0[b] - 1.0
            assert abs(log["bodies"][b]["dS"][k] - dS) <= 1e-12, (k, b)
    assert max(abs(v) for v in log["bodies"][0]["dS"]) > 0


def test_logged_run_stops_at_damage(lib):
    """A capsule set expanding is damaged by its first update: the log ends
    there, marked damaged, with the stretch beyond twice the rest length."""
    d = synth.pipe(24, 24, 24, 8.0, periodic_x=True, init="rest")
    c = np.array([12.2, 11.3, 11.6])
    X, Fc = synth.icosphere(1, 0.5, tuple(c), tilt=True)
    b = synth.Body(X, Fc, rigid=False, ca=0.05, r_ref=0.5, u_ref=0.02, v0=-2.4 * (X - c))
    w = synth.Workload("damage_log", d, [b], 0.8, 0.02, "f64", 5)
    lat = lib.from_workload(w)
    log = lib.campaign.log_run(lat, 10, 1, 0.02, 1.0)
    assert log["status"] == "damaged"
    assert log["bodies"][0]["stretch"][-1] >= 2.0
