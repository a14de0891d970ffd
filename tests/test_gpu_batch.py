"""Batching form on the GPU: independent instances advanced by one launch per
phase must compute exactly what each instance's own step computes (bitwise,
whatever the fluid launch shape), and match the oracle like the plain step.
"""
import sys

import numpy as np
import pytest

import oracle
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


def _small_instances(precision):
    """Uneven small instances: two bifurcations with capsules (one and two),
    a pipe with a rigid sphere, a pipe with a soft capsule, and a
    particle-free bifurcation."""
    return [synth.tiny_bifurcation(seed=0, precision=precision, n_bodies=2),
            synth.tiny_pipe(precision=precision, rigid=True),
            synth.tiny_bifurcation(seed=1, precision=precision, n_bodies=1),
            synth.tiny_pipe(precision=precision, rigid=False, nx=30),
            synth.tiny_bifurcation(seed=2, precision=precision, n_bodies=0)]


def _state(lat):
    rho, u = lat.fields()
    xs = [lat.body(b)[0] for b in range(len(lat.bodies))]
    return rho, u, xs


def _assert_same(lat_a, lat_b, what):
    import torch
    ra, ua, xa = _state(lat_a)
    rb, ub, xb = _state(lat_b)
    assert torch.equal(ra, rb) and torch.equal(ua, ub), what
    for p, q in zip(xa, xb):
        assert torch.equal(p, q), what


@pytest.mark.parametrize("shape", [None, (2, 128, 1, 0), (1, 64, 1, 64), (4, 256, 0, 0),
                                   (0, 64, 0, 0), (0, 128, 1, 64), (0, 256, 0, 128),
                                   (2, 64, 0, 64)])
def test_batch_equals_own_steps_bitwise(lib, shape):
    ws = _small_instances("f32")
    A = [lib.from_workload(w) for w in ws]
    B = [lib.from_workload(w) for w in ws]
    batch = lib.Batch(A)
    if shape is not None:
        batch.set_shape(*shape)
    _say(f"[batch] {len(ws)} instances, shape {batch.shape()}")
    batch.step(37)          # two graph chunks of 16 and five single steps
    for lat in B:
        lat.step(37)
    for lat in A + B:
        assert lat.sync(raise_on_stop=False) == 0
    for k, (a, b) in enumerate(zip(A, B)):
        _assert_same(a, b, f"instance {k}")
        assert a.info()["steps_done"] == 37


def test_batch_tracks_contexts_stepped_alone(lib):
    """Stepping one instance on its own, or adding a body, between batch
    steps is picked up by the next batch step."""
    ws = _small_instances("f64")[:3]
    A = [lib.from_workload(w) for w in ws]
    B = [lib.from_workload(w) for w in ws]
    batch = lib.Batch(A)
    batch.step(5)
    A[1].step(3)
    batch.step(4)
    extra = synth.tiny_pipe(precision="f64", rigid=True, body_radius=1.5).bodies[0]
    extra.x = extra.x + np.array([6.0, 0.0, 0.0])
    A[1].add_body(extra)
    batch.step(6)
    for k, lat in enumerate(B):
        lat.step(5)
        if k == 1:
            lat.step(3)
        lat.step(4)
        if k == 1:
            lat.add_body(extra)
        lat.step(6)
    for k, (a, b) in enumerate(zip(A, B)):
        assert a.sync(raise_on_stop=False) == 0
        _assert_same(a, b, f"instance {k}")


def test_batch_autotuner_keeps_results(lib):
    ws = _small_instances("f32")[:3]
    A = [lib.from_workload(w) for w in ws]
    B = [lib.from_workload(w) for w in ws]
    batch = lib.Batch(A)
    batch.step(3)
    tried = batch.tune(reps=3)
    _say(f"[batch] tuner tried {len(tried)} shapes, chose {batch.shape()}")
    assert len(tried) == 72   # FP32: V in {list, 1, 2, 4} x 3 block sizes x 6 fluid forms
    best = min(tried, key=lambda t: t["fluid_ms"])
    chosen = batch.shape()
    assert (chosen["bulk_v"], chosen["block"], chosen["mode"], chosen["per_xcd"]) == \
        (best["bulk_v"], best["block"], best["mode"], best["per_xcd"])
    batch.step(20)
    for lat in A:           # the tuned shape also serves each context's own step
        lat.step(5)
    for lat in B:
        lat.step(28)
    for k, (a, b) in enumerate(zip(A, B)):
        _assert_same(a, b, f"instance {k}")


@pytest.mark.parametrize("precision,shapes", [("f64", [(1, 64), (2, 128), (0, 64)]),
                                              ("f32", [(1, 64), (2, 256), (4, 128), (0, 128)]),
                                              ("f16s", [(2, 64), (4, 128), (8, 256), (0, 256)])])
def test_own_step_bitwise_for_every_launch_shape(lib, precision, shapes):
    """A context's own step gives the same bits for every supported launch
    shape of the stream-collide kernel."""
    w = synth.tiny_bifurcation(precision=precision, n_bodies=2)
    ref = lib.from_workload(w)
    ref.step(21)
    for v, blk in shapes:
        lat = lib.from_workload(w)
        lat.set_launch_shape(v, blk)
        lat.step(21)
        assert lat.sync(raise_on_stop=False) == 0
        _assert_same(lat, ref, f"shape {v}x{blk}")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_matches_oracle(lib, precision):
    tol = {"f64": 1e-12, "f32": 2e-5}[precision]
    ws = _small_instances(precision)[:2]
    A = [lib.from_workload(w) for w in ws]
    batch = lib.Batch(A)
    batch.step(30)
    for w, lat in zip(ws, A):
        assert lat.sync(raise_on_stop=False) == 0
        orc = oracle.from_workload(w)
        assert orc.step(30) == 0
        _, u_g = (t.cpu().numpy() for t in lat.fields())
        _, u_o = orc.fields()
        fl = w.domain.node_type != synth.SOLID
        e_u = np.abs(u_g[:, fl] - u_o[:, fl]).max() / np.abs(u_o[:, fl]).max()
        e_x = 0.0
        for b in range(len(w.bodies)):
            xg = lat.body(b)[0].cpu().numpy()
            xo = orc.body(b)[0]
            e_x = max(e_x, np.abs(xg - xo).max() / np.abs(xo - w.bodies[b].x).max())
        _say(f"[batch-oracle] {w.name} {precision}: e_u {e_u:.3e} e_x {e_x:.3e}")
        assert e_u <= tol and e_x <= tol


def test_batch_rejects_mixed_precision(lib):
    a = lib.from_workload(synth.tiny_pipe(precision="f32", with_body=False))
    b = lib.from_workload(synth.tiny_pipe(precision="f64", with_body=False))
    with pytest.raises(lib.LbmError):
        lib.Batch([a, b])
    with pytest.raises(lib.LbmError):
        lib.Batch([a, a])


def test_batching_form_instances_bitwise(lib):
    """The first four instances of the batching form at their full sizes
    (bifurcations of D = 24 to 48, 1-4 capsules each), in the tuned launch
    configuration: 12 batched steps equal 12 steps of each on its own."""
    ws = synth.batch_instances(n_instances=4, workers=4)
    A = [lib.from_workload(w) for w in ws]
    batch = lib.Batch(A)
    batch.tune(reps=2)
    _say(f"[batch] full-size instances, tuned shape {batch.shape()}")
    batch.step(12)
    for k, (w, a) in enumerate(zip(ws, A)):
        b = lib.from_workload(w)
        b.step(12)
        assert a.sync(raise_on_stop=False) == 0
        _assert_same(a, b, f"instance {k}")
        del b


def test_batch_of_one_and_of_fluid_only_instances(lib):
    """A batch of a single instance, and a batch whose instances carry no
    bodies (the IB phases have no work), equal their own steps bitwise."""
    for ws in ([synth.tiny_bifurcation(seed=4, precision="f32", n_bodies=1)],
               [synth.tiny_pipe(precision="f32", with_body=False),
                synth.tiny_bifurcation(seed=5, precision="f32", n_bodies=0)]):
        A = [lib.from_workload(w) for w in ws]
        B = [lib.from_workload(w) for w in ws]
        batch = lib.Batch(A)
        batch.step(19)
        for lat in B:
            lat.step(19)
        for k, (a, b) in enumerate(zip(A, B)):
            assert a.sync(raise_on_stop=False) == 0
            _assert_same(a, b, f"instance {k}")
