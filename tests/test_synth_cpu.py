"""Host-side checks of the synthetic workload generators: what the capsule
placement promises (inside the fluid, no overlap, off the stencil-switch
planes) and that the seeded draws are reproducible."""
import numpy as np
import pytest

import synth
from synth.mesh import off_switch_planes


def _check_placement(w, wall_clear=1.5, gap=2.0):
    sdf = w.domain.meta["sdf"]
    cs, rs = [], []
    for b in w.bodies:
        c = b.x.mean(0)
        r = np.linalg.norm(b.x - c, axis=1).max()
        # every vertex inside the fluid with the stated clearance
        assert sdf(c[None, :])[0] <= -(r + wall_clear) + 1e-9
        assert np.all(sdf(b.x) < 0.0)
        assert off_switch_planes(b.x, b.faces)
        cs.append(c)
        rs.append(r)
    for i in range(len(cs)):
        for j in range(i):
            assert np.linalg.norm(cs[i] - cs[j]) >= rs[i] + rs[j] + gap - 1e-9


@pytest.fixture(scope="module")
def precision_form():
    return synth.precision_form()


def test_precision_form_places_every_capsule(precision_form):
    w = precision_form
    assert len(w.bodies) == 16
    assert all(b.nv == 2562 for b in w.bodies)
    _check_placement(w)
    D = 48.0
    for b in w.bodies:
        c = b.x.mean(0)
        assert D <= c[0] <= 511 - D
        assert 0.3 * D / 2 - 1e-12 <= b.r_ref <= 0.8 * D / 2 + 1e-12
        assert 1e-3 <= b.ca <= 1e-1


def test_seeded_draws_are_reproducible():
    a, b = synth.tiny_bifurcation(seed=3, n_bodies=2), synth.tiny_bifurcation(seed=3, n_bodies=2)
    assert a.meta == b.meta
    for x, y in zip(a.bodies, b.bodies):
        np.testing.assert_array_equal(x.x, y.x)
        assert x.ca == y.ca


@pytest.mark.parametrize("n", [1, 2])
def test_tiny_bifurcation_placement(n):
    _check_placement(synth.tiny_bifurcation(n_bodies=n), wall_clear=0.0, gap=0.0)


def test_bifurcation_capsule_is_off_switch_planes():
    w = synth.bifurcation_capsule()
    assert len(w.bodies) == 1 and w.bodies[0].nv == 2562
    assert off_switch_planes(w.bodies[0].x, w.bodies[0].faces)


def test_smooth_junction_has_a_flat_wall():
    """The smooth junction replaces the sharp apex between the daughters by
    a flat wall normal to the main axis: across a band around the symmetry
    plane the first solid node beyond the junction sits at one x, one
    daughter radius past the sharp apex; the sharp junction's apex is a
    V (the first solid x grows off the symmetry plane)."""
    first = {}
    for j in ("sharp", "smooth"):
        d = synth.bifurcation(256, 128, 40, 32.0, 0.8, 60.0, 4.0, u_max=0.02, junction=j)
        nt = d.node_type.reshape(40, 128, 256)
        xs = []
        for dy in range(-6, 7):
            row = nt[20, 64 + dy, 129:]
            xs.append(129 + int(np.flatnonzero(row == synth.SOLID)[0]))
        first[j] = xs
        assert np.all((d.link_q >= 0) & (d.link_q <= 1))
    assert len(set(first["smooth"])) == 1
    # (the sharp apex is rounded by the 4 lu fillet near the plane)
    assert first["sharp"][6] < first["sharp"][0] and first["sharp"][6] < first["sharp"][-1]
    # the flat wall lies about one daughter radius (12.8) past the sharp apex
    assert 9 <= first["smooth"][6] - first["sharp"][6] <= 14


def test_capsule_trains_are_placed_as_stated():
    """Three bodies on one line at 1.16 D, 2.01 D, 2.86 D from the inlet;
    soft capsules of radius D/3, rigid spheres of half that; all in the
    fluid and off the stencil-switch planes; seeded offset reproducible."""
    for train, kinds in synth.TRAIN_KINDS.items():
        w = synth.capsule_train(train)
        D = 32.0
        sdf = w.domain.meta["sdf"]
        for k, (b, kind) in enumerate(zip(w.bodies, kinds)):
            c = b.x.mean(0)
            assert abs(c[0] - (1.16 + 0.85 * k) * D) < 1e-9
            r = np.linalg.norm(b.x - c, axis=1).max()
            assert abs(r - (D / 3 if kind == "soft" else D / 6)) < 1e-9
            assert b.rigid == (kind == "rigid")
            assert np.all(sdf(b.x) < 0.0) and off_switch_planes(b.x, b.faces)
        assert w.meta["offset"] == synth.capsule_train(train).meta["offset"]
