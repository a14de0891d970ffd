"""The marker order does not depend on the order in which the caller lists a
capsule's faces (or rotates their vertex lists): the library sorts each
body's faces into marker slots by the position of their stencil bases along
the Hilbert curve (k_bin_faces, when a body is added and every 512 steps),
so a block of 64 markers is a patch of neighbouring faces whatever the input
order.

Checked with the faces of every body randomly permuted (the same mesh):
parity with the oracle given the same permuted mesh at the usual bars (two
soft capsules in the small bifurcation, FP64 and FP32); bitwise agreement
with the run on the original order (the library keeps its faces in a
canonical order, and the forcing does not depend on the marker order); a
body above the LDS capacity of the sort (a rigid sphere of 20480 faces,
sorted in global memory); and, on the full bifurcation with the 2562-vertex
capsule, the FP64 run past two re-sorts bit for bit against the original
order and the FP32 step time within 10 % of the original order's."""
import copy
import sys
import time

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


def _permuted(w, seed):
    """The same meshes with the faces in a random order, each face's vertex
    list turned by a random cyclic shift (orientation kept)."""
    rng = np.random.default_rng(seed)
    w2 = copy.deepcopy(w)
    for b in w2.bodies:
        F = b.faces[rng.permutation(b.nf)]
        r = rng.integers(0, 3, size=b.nf)
        F = np.stack([F[np.arange(b.nf), (r + k) % 3] for k in range(3)], 1)
        b.faces = np.ascontiguousarray(F, dtype=np.int32)
    return w2


def _errors(lat, ref_u, ref_x, w):
    rho, u = (t.cpu().numpy() for t in lat.fields())
    fl = w.domain.node_type != synth.SOLID
    e_u = np.abs(u[:, fl] - ref_u[:, fl]).max() / np.abs(ref_u[:, fl]).max()
    e_x = 0.0
    for b in range(len(w.bodies)):
        disp = np.abs(ref_x[b] - w.bodies[b].x).max()
        e_x = max(e_x, np.abs(lat.body(b)[0].cpu().numpy() - ref_x[b]).max() / disp)
    return e_u, e_x


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_permuted_faces_match_the_oracle(lib, precision):
    w = synth.tiny_bifurcation(precision=precision, n_bodies=2)
    wp = _permuted(w, 5)
    steps = 30
    _say(f"[binning] two capsules, permuted faces, {precision}, {steps} steps")
    lat = lib.from_workload(wp, precision=precision)
    lat.step(steps)
    assert lat.sync(raise_on_stop=False) == 0
    orc = oracle.from_workload(wp)
    assert orc.step(steps) == 0
    ref_u = orc.fields()[1]
    ref_x = [orc.body(b)[0] for b in range(len(wp.bodies))]
    e_u, e_x = _errors(lat, ref_u, ref_x, wp)
    _say(f"    vs oracle e_u {e_u:.3e} e_x {e_x:.3e}")
    assert e_u <= TOL[precision] and e_x <= TOL[precision]
    # the original order on the GPU
    lo = lib.from_workload(w, precision=precision)
    lo.step(steps)
    assert lo.sync(raise_on_stop=False) == 0
    u_o = lo.fields()[1].cpu().numpy()
    x_o = [lo.body(b)[0].cpu().numpy() for b in range(len(w.bodies))]
    e_u2, e_x2 = _errors(lat, u_o, x_o, w)
    _say(f"    vs original order e_u {e_u2:.3e} e_x {e_x2:.3e}")
    # the library's own face order is canonical: the same run bit for bit
    assert e_u2 == 0.0 and e_x2 == 0.0


def _big_sphere_workload(precision):
    """A pipe D = 56 on a 72x60x60 grid with one rigid sphere of radius 20
    meshed with 20480 faces (icosphere subdivision 5, edges ~0.7 dx)."""
    u_max, tau = 0.02, 0.8
    dom = synth.pipe(72, 60, 60, 28.0, u_max=u_max, tau=tau, init="poiseuille")
    X, F = synth.icosphere(5, 20.0, (30.0, 29.5, 29.5), tilt=True)
    body = synth.Body(X, F, rigid=True, rho_ratio=1.1, r_ref=20.0, u_ref=u_max)
    return synth.Workload("pipe_big_sphere", dom, [body], tau, u_max, precision, 10)


def test_body_sorted_in_global_memory(lib):
    w = _big_sphere_workload("f64")
    assert w.bodies[0].nf == 20480
    wp = _permuted(w, 9)
    steps = 12
    _say(f"[binning] 20480-face sphere, permuted faces, f64, {steps} steps")
    lat = lib.from_workload(wp, precision="f64")
    lat.step(steps)
    assert lat.sync(raise_on_stop=False) == 0
    orc = oracle.from_workload(wp)
    assert orc.step(steps) == 0
    e_u, e_x = _errors(lat, orc.fields()[1], [orc.body(0)[0]], wp)
    _say(f"    vs oracle e_u {e_u:.3e} e_x {e_x:.3e}")
    assert e_u <= TOL["f64"] and e_x <= TOL["f64"]


def _released(P, w, precision, precursor):
    lat = P.Lattice(w.domain, w.tau, w.u_max, precision)
    lat.step(precursor)
    lat.sync()
    lat.add_body(w.bodies[0])
    return lat


def _step_time(P, w, steps, reps=3):
    lat = _released(P, w, "f32", 200)
    lat.step(100)
    lat.sync()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        lat.step(steps)
        lat.sync()
        best = min(best, time.perf_counter() - t0)
    return best / steps


def test_permuted_faces_run_as_fast(lib):
    w = synth.bifurcation_capsule(precision="f32")
    wp = _permuted(w, 7)
    _say("[binning] full bifurcation, step time, original vs permuted faces")
    t_o = _step_time(lib, w, 1024)
    t_p = _step_time(lib, wp, 1024)
    _say(f"    original {t_o * 1e6:.2f} us/step, permuted {t_p * 1e6:.2f} us/step")
    assert t_p <= 1.1 * t_o


def test_permuted_faces_full_size_f64(lib):
    """Past two re-sorts of the marker order (1100 steps after the release)."""
    w = synth.bifurcation_capsule(precision="f64")
    wp = _permuted(w, 7)
    steps = 1100
    _say(f"[binning] full bifurcation, f64, original vs permuted faces, {steps} steps")
    lo, lp = _released(lib, w, "f64", 200), _released(lib, wp, "f64", 200)
    for lat in (lo, lp):
        lat.step(steps)
        assert lat.sync(raise_on_stop=False) == 0
    e_u, e_x = _errors(lp, lo.fields()[1].cpu().numpy(), [lo.body(0)[0].cpu().numpy()], w)
    _say(f"    permuted vs original e_u {e_u:.3e} e_x {e_x:.3e}")
    assert e_u == 0.0 and e_x == 0.0
