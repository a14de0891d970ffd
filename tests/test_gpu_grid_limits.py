"""The kernels index nodes with 32-bit integers (padded index x + px (y + ny z),
px = nx rounded up to a multiple of 8, with one guard plane on each side in
z).  A grid whose node count is allowed but whose padded count with the
guard planes reaches 2^31 must be refused at creation, before anything is
allocated on the device."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_padded_index_limit_is_refused():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2207_06043_amd as P
    P.load_library()
    nx, ny, nz = 1, 16384, 16400
    # nx ny nz = 268,697,600 nodes pass the plain size check; padded to
    # px = 8 with two guard planes they exceed 2^31
    assert nx * ny * nz < (1 << 31) - (1 << 20)
    assert 8 * ny * (nz + 2) >= 1 << 31
    d = synth.periodic_box(nx, ny, nz)
    with pytest.raises(P.LbmError) as e:
        P.Lattice(d, 0.8, 0.0, "f32")
    assert "grid too large" in str(e.value)
