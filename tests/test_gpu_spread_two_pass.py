"""The spread in two passes, the atomics-free alternative: each marker block
stores its box of fixed-point sums (accumulated in LDS), and an owner pass
adds, for every node, the boxes of all chunks that hold it, in chunk order,
with plain stores (LBM_SPREAD_TWO_PASS=1 at creation).  The default spread
adds each block's box sums with 64-bit integer atomics.  Both add the same
integers, so every case must agree bit for bit; the step times of the two
on the full bifurcation are printed (the faster one is the default)."""
import os
import sys
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


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


def _lattice(P, w, precision, two_pass):
    old = os.environ.get("LBM_SPREAD_TWO_PASS")
    os.environ["LBM_SPREAD_TWO_PASS"] = "1" if two_pass else "0"
    try:
        return P.Lattice(w.domain, w.tau, w.u_max, precision)
    finally:
        if old is None:
            del os.environ["LBM_SPREAD_TWO_PASS"]
        else:
            os.environ["LBM_SPREAD_TWO_PASS"] = old


def _run(P, w, precision, steps, two_pass, precursor=0, timed=0):
    lat = _lattice(P, w, precision, two_pass)
    if precursor:
        lat.step(precursor)
        lat.sync()
    for b in w.bodies:
        lat.add_body(b)
    lat.step(steps)
    st = lat.sync(raise_on_stop=False)
    dt = None
    if timed:
        best = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            lat.step(timed)
            lat.sync()
            best = min(best, time.perf_counter() - t0)
        dt = best / timed
    rho, u = (t.cpu().numpy() for t in lat.fields())
    f = lat.force().cpu().numpy()
    xs = [lat.body(b)[0].cpu().numpy() for b in range(len(w.bodies))]
    return st, rho, u, f, xs, dt


def _same(a, b):
    assert a[0] == b[0] == 0
    for k in (1, 2, 3):
        assert np.array_equal(a[k], b[k])
    for xa, xb in zip(a[4], b[4]):
        assert np.array_equal(xa, xb)


def test_two_pass_equals_atomics_two_capsules(lib):
    w = synth.tiny_bifurcation(precision="f64", n_bodies=2)
    _say("[spread] two capsules f64, 30 steps: two-pass vs atomics")
    _same(_run(lib, w, "f64", 30, True), _run(lib, w, "f64", 30, False))


def test_two_pass_equals_atomics_across_a_periodic_face(lib):
    d = synth.periodic_box(40, 20, 20, body_force=(2e-6, 0.0, 0.0))
    X1, F1 = synth.icosphere(2, 3.0, (0.5, 9.5, 9.5), tilt=True)
    X2, F2 = synth.icosphere(2, 3.0, (20.0, 0.2, 19.6), tilt=True)
    bodies = [synth.Body(X1, F1, rigid=True, rho_ratio=1.1, r_ref=3.0, u_ref=0.01),
              synth.Body(X2, F2, rigid=False, ca=0.05, r_ref=3.0, u_ref=0.01)]
    w = synth.Workload("periodic_bodies", d, bodies, 0.8, 0.01, "f64", 30)
    _say("[spread] periodic box, bodies on the periodic faces, f64, 30 steps")
    _same(_run(lib, w, "f64", 30, True), _run(lib, w, "f64", 30, False))


def test_two_pass_equals_atomics_full_bifurcation(lib):
    w = synth.bifurcation_capsule(precision="f32")
    _say("[spread] full bifurcation f32, 600 steps after 300, then timed")
    a = _run(lib, w, "f32", 600, True, precursor=300, timed=1024)
    b = _run(lib, w, "f32", 600, False, precursor=300, timed=1024)
    _say(f"    step: two-pass {a[5] * 1e6:.2f} us, atomics {b[5] * 1e6:.2f} us")
    # the timed steps continue both runs identically
    _same(a, b)
