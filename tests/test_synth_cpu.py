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
