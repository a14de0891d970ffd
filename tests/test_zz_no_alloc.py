"""The allocation-free spread (ib_spread_noalloc) against ib_spread, through
the C ABI: same inputs, bitwise the same force field, on two calls in a row
(the second with a smaller lattice and fewer points, so the scratch left by
the first must not leak into it), plus the size limit."""
import sys

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


def _points(rng, n, nx, cy, cz, rmax):
    r = rng.uniform(0, rmax, n)
    t = rng.uniform(0, 2 * np.pi, n)
    return np.stack([rng.uniform(-3, nx + 3, n), cy + r * np.cos(t), cz + r * np.sin(t)], 1)


def _case(lib, lat, rng, pts, N):
    import torch
    dev = lat.device
    n = pts.shape[0]
    F = torch.from_numpy(rng.normal(size=(n, 3)) * 1e-3).to(dev)
    c = torch.from_numpy(rng.uniform(0.1, 1.0, n)).to(dev)
    P = torch.from_numpy(pts).to(dev)
    base = torch.from_numpy(rng.normal(size=(3, N)) * 1e-4).to(dev)  # the call adds into d_fib
    ref = lat.ib_spread(P, F, c, base.clone())
    out = base.clone()
    lat.ib_spread_noalloc(P, F, c, out)
    lat.sync()
    return ref.cpu().numpy(), out.cpu().numpy(), base.cpu().numpy()


def test_noalloc_spread_equals_ib_spread(lib):
    rng = np.random.default_rng(11)
    # first call: 24 x 16 x 16 periodic pipe, 400 points
    d1 = synth.pipe(24, 16, 16, 6.5, periodic_x=True, init="rest")
    lat1 = lib.from_workload(synth.Workload("noalloc_a", d1, [], 0.8, 0.0, "f64", 0))
    _say("[noalloc] call 1: 24x16x16 pipe, 400 points")
    ref, out, base = _case(lib, lat1, rng, _points(rng, 400, 24, 7.5, 7.5, 6.3), d1.n_nodes)
    assert np.abs(ref - base).max() > 0  # the spread added something
    assert np.array_equal(ref, out)
    # second call: a smaller lattice (16 x 14 x 14) and fewer points
    d2 = synth.pipe(16, 14, 14, 5.6, periodic_x=True, init="rest")
    lat2 = lib.from_workload(synth.Workload("noalloc_b", d2, [], 0.8, 0.0, "f32", 0))
    _say("[noalloc] call 2: 16x14x14 pipe, 37 points")
    ref, out, base = _case(lib, lat2, rng, _points(rng, 37, 16, 6.5, 6.5, 5.5), d2.n_nodes)
    assert np.abs(ref - base).max() > 0
    assert np.array_equal(ref, out)
    # no points: d_fib unchanged
    import torch
    z = torch.from_numpy(rng.normal(size=(3, d2.n_nodes))).to(lat2.device)
    z0 = z.clone()
    e = torch.zeros(0, 3, dtype=torch.float64, device=lat2.device)
    lat2.ib_spread_noalloc(e, e, torch.zeros(0, dtype=torch.float64, device=lat2.device), z)
    lat2.sync()
    assert torch.equal(z, z0)


def test_noalloc_spread_refuses_lattices_beyond_the_scratch(lib):
    import torch
    from paper_2207_06043_amd import LbmError
    # 136 x 128 x 128 = 2,228,224 padded nodes > 2^21
    d = synth.periodic_box(136, 128, 128)
    lat = lib.from_workload(synth.Workload("noalloc_big", d, [], 0.8, 0.0, "f16s", 0))
    _say("[noalloc] size limit")
    pts = torch.tensor([[5.2, 6.1, 4.7]], dtype=torch.float64, device=lat.device)
    F = torch.tensor([[1e-3, 0.0, 0.0]], dtype=torch.float64, device=lat.device)
    c = torch.ones(1, dtype=torch.float64, device=lat.device)
    fib = torch.zeros(3, d.n_nodes, dtype=torch.float64, device=lat.device)
    with pytest.raises(LbmError, match="scratch holds at most"):
        lat.ib_spread_noalloc(pts, F, c, fib)
    # the context is still usable
    ref = lat.ib_spread(pts, F, c)
    assert float(ref.abs().sum()) > 0
