"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (the velocity table, the north-wall Zou-He block), closed-form
moment identities, polynomial exactness of the interpolation rules, library
routines (least squares, convex hull), invariances, and energy gradients.
"""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]
    return np.array(rows, dtype=np.float64)


# ------------------------------------------------------------ lattice (Eq. e_i)
def test_velocity_set_matches_printed_table():
    e, w = oracle.lattice()
    printed = _table("d3q19_velocity_set.txt").astype(int)
    assert np.array_equal(e.T, printed)
    assert np.array_equal(synth.D3Q19_DIRS.T, printed)
    assert np.allclose(w[0], 1 / 3) and np.allclose(w[1:7], 1 / 18) and np.allclose(w[7:], 1 / 36)


def test_lattice_isotropy():
    e, w = oracle.lattice()
    e = e.astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ e).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), np.eye(3) / 3, atol=1e-16)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, e, e, e)).max() < 1e-16
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), iso, atol=1e-16)


# ------------------------------------------------------ equilibrium and forcing
@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    e, _ = oracle.lattice()
    rho, u = rng.uniform(0.8, 1.2), rng.uniform(-0.1, 0.1, 3)
    f = oracle.feq(rho, u)
    assert abs(f.sum() - rho) < 1e-15
    assert np.abs(f @ e - rho * u).max() < 1e-16
    Pi = np.einsum("i,ia,ib->ab", f, e, e)
    assert np.abs(Pi - (rho / 3 * np.eye(3) + rho * np.outer(u, u))).max() < 1e-15


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 1.7])
def test_forcing_moments(tau):
    rng = np.random.default_rng(int(tau * 100))
    e, _ = oracle.lattice()
    u, F = rng.uniform(-0.1, 0.1, 3), rng.uniform(-1e-3, 1e-3, 3)
    G = oracle.guo(tau, u, F)
    k = 1 - 1 / (2 * tau)
    assert abs(G.sum()) < 1e-18
    assert np.abs(G @ e - k * F).max() < 1e-18
    Pi = np.einsum("i,ia,ib->ab", G, e, e)
    assert np.abs(Pi - k * (np.outer(u, F) + np.outer(F, u))).max() < 1e-18


# ------------------------------------------------------------- Zou-He (Eq. extbound)
def _near_eq(rng):
    return oracle.feq(1.0 + rng.uniform(-0.02, 0.02), rng.uniform(-0.05, 0.05, 3)) * (1 + rng.uniform(-0.05, 0.05, 19))


@pytest.mark.parametrize("face", range(6))
def test_zouhe_velocity_face_moments(face):
    rng = np.random.default_rng(face)
    e, _ = oracle.lattice()
    uw = rng.uniform(-0.05, 0.05, 3)
    f, rho = oracle.zouhe(_near_eq(rng), face, 0, uw)
    assert abs(f.sum() - rho) < 1e-15
    assert np.abs(f @ e - rho * uw).max() < 2e-16


@pytest.mark.parametrize("face", range(6))
def test_zouhe_density_face_moments(face):
    rng = np.random.default_rng(10 + face)
    e, _ = oracle.lattice()
    rhow = 1.0 + rng.uniform(-0.01, 0.01)
    f, rho = oracle.zouhe(_near_eq(rng), face, 1, rho_w=rhow)
    assert rho == rhow
    assert abs(f.sum() - rhow) < 1e-15
    m = f @ e
    axis = face // 2
    tang = [a for a in range(3) if a != axis]
    assert np.abs(m[tang]).max() < 2e-16  # tangential velocity imposed zero


def test_zouhe_matches_printed_north_wall_block():
    """The printed north-wall block (z = z_max, inward normal -z), read in its
    own population order (golden map) and with the wall density on the 1/6
    terms, must give the same populations as the general-face rule."""
    e, _ = oracle.lattice()
    m = _table("zouhe_north_wall.txt").astype(int)
    vec2idx = {tuple(v): i for i, v in enumerate(e)}
    P = {int(r[0]): vec2idx[tuple(r[1:])] for r in m}  # printed index -> our index
    rng = np.random.default_rng(7)
    f0 = _near_eq(rng)
    ux, uy, uz = rng.uniform(-0.05, 0.05, 3)
    ours, rho_g = oracle.zouhe(f0, 5, 0, (ux, uy, uz))
    g = lambda k: f0[P[k]]
    rho = (g(0) + g(1) + g(2) + g(3) + g(4) + g(7) + g(8) + g(13) + g(14)
           + 2 * (g(5) + g(9) + g(11) + g(16) + g(18))) / (uz + 1)
    Nzx = 0.5 * (g(1) + g(7) + g(13) - (g(2) + g(14) + g(8))) - rho * ux / 3
    Nzy = 0.5 * (g(3) + g(7) + g(14) - (g(4) + g(13) + g(8))) - rho * uy / 3
    printed = {6: g(5) - rho * uz / 3,
               15: g(16) + rho / 6 * (-uz + ux) - Nzx,
               10: g(9) + rho / 6 * (-uz - ux) + Nzx,
               17: g(18) + rho / 6 * (-uz + uy) - Nzy,
               12: g(11) + rho / 6 * (-uz - uy) + Nzy}
    assert abs(rho - rho_g) < 1e-15
    for k, v in printed.items():
        assert abs(ours[P[k]] - v) < 1e-15, k


# ----------------------------------------------------- BFL (Eq. bbouzidi)
@pytest.mark.parametrize("q", [0.0, 0.1, 0.25, 0.4999, 0.5, 0.6, 0.83, 1.0])
def test_bfl_is_quadratic_interpolation(q):
    """q < 1/2 interpolates f*_i at s = 2q-1 through s = 0, -1, -2; q >= 1/2
    interpolates the returning population at s = 0 through the bounced value
    at s = 2q-1 and the opposite populations at s = -1, -2.  Both must be
    exact for any quadratic."""
    rng = np.random.default_rng(int(q * 1e4))
    c = rng.normal(size=3)
    P = lambda s: c[0] + c[1] * s + c[2] * s * s
    if q < 0.5:
        got = oracle.bfl(q, P(0), P(-1), P(-2), 0.0, 0.0)
        assert abs(got - P(2 * q - 1)) < 1e-13
    else:
        got = oracle.bfl(q, P(2 * q - 1), 0.0, 0.0, P(-1), P(-2))
        assert abs(got - P(0)) < 1e-13


@pytest.mark.parametrize("q", [0.2, 0.45, 0.5, 0.7, 0.95])
def test_bfl_fallbacks_are_linear_interpolation(q):
    rng = np.random.default_rng(int(q * 100))
    c = rng.normal(size=2)
    P = lambda s: c[0] + c[1] * s
    if q < 0.5:
        assert abs(oracle.bfl(q, P(0), P(-1), 123.0, 0, 0, True, False) - P(2 * q - 1)) < 1e-14
        assert oracle.bfl(q, 0.7, 1.0, 2.0, 0, 0, False, False) == 0.7
    else:
        assert abs(oracle.bfl(q, P(2 * q - 1), 0, 0, P(-1), 9.0, False, False) - P(0)) < 1e-14


def test_bfl_halfway_and_continuity():
    vals = (0.31, 0.29, 0.27, 0.33, 0.35)
    assert oracle.bfl(0.5, *vals) == pytest.approx(0.31, abs=1e-16)
    lo = oracle.bfl(0.5 - 1e-9, *vals)
    hi = oracle.bfl(0.5 + 1e-9, *vals)
    assert abs(lo - hi) < 1e-8


def test_pipe_link_fraction_lies_on_wall():
    d = synth.pipe(8, 20, 20, 8.0).__dict__
    e = synth.D3Q19_DIRS
    n = d["link_node"]
    x, y, z = n % 8, (n // 8) % 20, n // 160
    p = np.stack([x, y, z], 1) + d["link_q"][:, None] * e[d["link_dir"]]
    r = np.hypot(p[:, 1] - 9.5, p[:, 2] - 9.5)
    assert np.abs(r - 8.0).max() < 1e-12


# -------------------------------------------------- conservation (periodic box)
def test_periodic_box_mass_and_momentum_budget():
    """With a uniform force g on every node, each step adds exactly g per node
    to the total momentum (Guo forcing) and leaves the mass unchanged."""
    g = np.array([1e-5, -2e-6, 3e-6])
    d = synth.periodic_box(6, 5, 4, body_force=g)
    rng = np.random.default_rng(3)
    d.init_rho = 1 + 0.01 * rng.standard_normal(d.n_nodes)
    d.init_u = 0.01 * rng.standard_normal(3 * d.n_nodes)
    s = oracle.OracleSim(d, tau=0.9, threads=1)
    e, _ = oracle.lattice()
    f0 = s.populations()
    M0, P0 = f0.sum(), (e.T @ f0).sum(axis=1)
    s.step(5)
    f1 = s.populations()
    assert abs(f1.sum() - M0) < 1e-12
    assert np.abs((e.T @ f1).sum(axis=1) - (P0 + 5 * d.n_nodes * g)).max() < 1e-13


# ------------------------------------------------------ MLS (Eqs. uLag, l2norm, intKernel)
def _pipe_sim():
    d = synth.pipe(12, 12, 12, 4.6, periodic_x=True, init="rest")
    return d, oracle.OracleSim(d, tau=0.8, threads=1)


@pytest.mark.parametrize("seed", range(6))
def test_mls_reproduces_linear_fields(seed):
    d, s = _pipe_sim()
    rng = np.random.default_rng(seed)
    # points inside the pipe, some close to the wall (excluded solid nodes)
    r = rng.uniform(0, 4.4)
    t = rng.uniform(0, 2 * np.pi)
    p = np.array([rng.uniform(0, 11), 5.5 + r * np.cos(t), 5.5 + r * np.sin(t)])
    ok, node, psi = s.mls_point(p)
    assert ok
    a, G = rng.normal(), rng.normal(size=3)
    x = np.stack([node % 12, (node // 12) % 12, node // 144], 1).astype(float)
    # unwrap periodic x relative to p
    x[:, 0] += 12 * np.round((p[0] - x[:, 0]) / 12)
    val = a + (x - p) @ G
    m = node >= 0
    assert abs(psi[m, 0].sum() - 1) < 1e-13                      # partition of unity
    assert np.abs(psi[m, 0] @ (x[m] - p)).max() < 1e-13          # first moments
    assert abs(psi[m, 0] @ val[m] - a) < 1e-12                   # value of a linear field
    assert np.abs(psi[m, 1:].T @ val[m] - G).max() < 1e-12       # its gradient
    assert np.all(psi[~m] == 0)


def test_mls_weights_equal_weighted_least_squares():
    """phi_k from the oracle equals the weighted least-squares solution from a
    library solver with the kernel W = exp(-(r/0.3)^2), r = |x_k - x| / 2.6."""
    d = synth.periodic_box(8, 8, 8)
    s = oracle.OracleSim(d, tau=0.8, threads=1)
    rng = np.random.default_rng(11)
    for _ in range(5):
        p = rng.uniform(2, 5, 3)
        ok, node, psi = s.mls_point(p)
        b = np.floor(p + 0.5)
        offs = np.array([[k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1] for k in range(27)], float)
        xk = b + offs
        r = np.linalg.norm(xk - p, axis=1) / 2.6
        W = np.where(r <= 1, np.exp(-(r / 0.3) ** 2), 0.0)
        P = np.hstack([np.ones((27, 1)), xk - p])
        sw = np.sqrt(W)[:, None]
        # phi solves min sum W (p^T a - u)^2 for every u: rows of the pseudo-inverse
        pinv = np.linalg.pinv(sw * P) * sw.T
        assert np.abs(pinv[0] - psi[:, 0]).max() < 1e-11
        assert np.abs(pinv[1:] - psi[:, 1:].T).max() < 1e-10


def test_spread_conserves_force_and_torque_and_is_adjoint():
    d, s = _pipe_sim()
    rng = np.random.default_rng(5)
    n = 40
    r = rng.uniform(0, 4.0, n)
    t = rng.uniform(0, 2 * np.pi, n)
    pts = np.stack([rng.uniform(2, 9, n), 5.5 + r * np.cos(t), 5.5 + r * np.sin(t)], 1)
    F = rng.normal(size=(n, 3)) * 1e-3
    c = rng.uniform(0.2, 1.0, n)
    fib = s.ib_spread(pts, F, c)
    assert np.abs(fib.sum(axis=1) - (c[:, None] * F).sum(0)).max() < 1e-15
    N = d.n_nodes
    idx = np.arange(N)
    X = np.stack([idx % 12, (idx // 12) % 12, idx // 144], 1).astype(float)
    tq_grid = np.cross(X, fib.T).sum(0)
    tq_pts = np.cross(pts, c[:, None] * F).sum(0)
    assert np.abs(tq_grid - tq_pts).max() < 1e-13
    u = rng.normal(size=(3, N))
    lhs = np.sum(s.ib_interpolate(pts, u) * (c[:, None] * F))
    rhs = np.sum(u * fib)
    assert abs(lhs - rhs) < 1e-14


# ------------------------------------------------------------- membrane
def _capsule_sim(subdiv=2, rigid=False):
    d = synth.periodic_box(16, 16, 16)
    X, Fc = synth.icosphere(subdiv, 4.0, (7.6, 8.1, 7.9))
    b = synth.Body(X, Fc, rigid=rigid, ca=0.05, eb=0.01, rho_ratio=1.1, r_ref=4.0, u_ref=0.02)
    return b, oracle.OracleSim(d, tau=0.8, u_max=0.02, bodies=[b], threads=1)


def test_mesh_volume_and_area_match_convex_hull():
    from scipy.spatial import ConvexHull
    b, s = _capsule_sim(3)
    hull = ConvexHull(b.x)
    dg = s.body_diag(0)
    assert abs(dg["V0"] - hull.volume) < 1e-10
    assert abs(dg["S0"] - hull.area) < 1e-10


@pytest.mark.parametrize("which", [1, 2, 4])
def test_membrane_zero_at_rest(which):
    b, s = _capsule_sim()
    E, F = s.membrane(0, b.x, which)
    assert abs(E) < 1e-20 and np.abs(F).max() < 1e-13


@pytest.mark.parametrize("which", [1, 2, 4])
def test_membrane_force_is_minus_energy_gradient(which):
    b, s = _capsule_sim()
    rng = np.random.default_rng(which)
    x = b.x + rng.normal(scale=0.15, size=b.x.shape)
    _, F = s.membrane(0, x, which)
    h = 1e-6
    for v in rng.choice(len(x), 12, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[v, a] += h
            xm[v, a] -= h
            fd = -(s.membrane(0, xp, which)[0] - s.membrane(0, xm, which)[0]) / (2 * h)
            assert abs(fd - F[v, a]) <= 1e-7 * max(1e-3, np.abs(F).max()), (v, a, fd, F[v, a])


@pytest.mark.parametrize("which", [1, 2, 4])
def test_membrane_forces_have_no_net_force_or_torque(which):
    b, s = _capsule_sim()
    rng = np.random.default_rng(10 + which)
    x = b.x + rng.normal(scale=0.2, size=b.x.shape)
    _, F = s.membrane(0, x, which)
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-12 * scale * len(x)
    assert np.abs(np.cross(x, F).sum(0)).max() < 1e-11 * scale * len(x)


# -------------------------------------------------- hydrodynamic probes (S7)
def _probe_box(rho, u, subdiv=2):
    d = synth.periodic_box(20, 20, 20)
    d.init_rho = rho
    d.init_u = u
    X, Fc = synth.icosphere(subdiv, 4.0, (9.7, 10.2, 9.9))
    b = synth.Body(X, Fc, rigid=True, rho_ratio=1.1, r_ref=4.0)
    return b, oracle.OracleSim(d, tau=0.8, bodies=[b], threads=1)


def _grid(n=20):
    i = np.arange(n ** 3)
    return np.stack([i % n, (i // n) % n, i // (n * n)], 1).astype(float)


def test_probe_forces_vanish_for_uniform_pressure_and_rigid_motion():
    X = _grid()
    U, Om = np.array([0.01, -0.02, 0.005]), np.array([1e-3, 2e-3, -1e-3])
    u = (U + np.cross(Om, X - 10.0)).T.ravel()
    b, s = _probe_box(np.full(len(X), 1.02), u)
    F = s.body_hydro(0)
    assert np.abs(F).max() < 1e-14


def test_probe_forces_closed_form_for_linear_density_and_shear():
    """rho = 1 + a.x (p = rho/3) with the uniform shear u = (gamma z, 0, 0):
    MLS reproduces both exactly, so per face
    F = 2.4 (a.n) [-n/3 + nu gamma S n] A, S = e_x e_z^T + e_z e_x^T."""
    X = _grid()
    a = np.array([2e-4, -1e-4, 3e-4])
    gam = 1e-3
    rho = 1.0 + (X - 10.0) @ a
    u = np.zeros((3, len(X)))
    u[0] = gam * (X[:, 2] - 10.0)
    b, s = _probe_box(rho, u.ravel())
    F = s.body_hydro(0)
    nu = (0.8 - 0.5) / 3
    S = np.zeros((3, 3))
    S[0, 2] = S[2, 0] = 1.0
    x = b.x
    A_ = 0.5 * np.cross(x[b.faces[:, 1]] - x[b.faces[:, 0]], x[b.faces[:, 2]] - x[b.faces[:, 0]])
    area = np.linalg.norm(A_, axis=1)
    n = A_ / area[:, None]
    an = n @ a
    expect = 2.4 * an[:, None] * (-n / 3 + nu * gam * (n @ S.T)) * area[:, None]
    assert np.abs(F - expect).max() < 1e-15


# ---------------------------------------------------- motion (S8)
def _uniform_flow_body(rigid):
    U = np.array([0.02, -0.01, 0.015])
    d = synth.periodic_box(24, 24, 24)
    d.init_u = np.repeat(U[:, None], d.n_nodes, 1).ravel()
    X, Fc = synth.icosphere(2, 4.0, (11.3, 12.1, 11.7))
    b = synth.Body(X, Fc, rigid=rigid, ca=0.05, eb=0.01, rho_ratio=1.1, r_ref=4.0, u_ref=0.02,
                   v0=np.repeat(U[None, :], len(X), 0))
    return U, b, oracle.OracleSim(d, tau=0.8, u_max=0.02, bodies=[b], threads=2)


@pytest.mark.parametrize("rigid", [False, True])
def test_body_in_uniform_flow_translates_undeformed(rigid):
    U, b, s = _uniform_flow_body(rigid)
    s.step(10)
    x, v = s.body(0)
    assert np.abs(x - (b.x + 10 * U)).max() < 1e-12
    assert np.abs(v - U).max() < 1e-13
    rho, u = s.fields()
    assert np.abs(u - U[:, None]).max() < 1e-13
    assert np.abs(s.force()).max() < 1e-14


def test_damage_stops_the_computation():
    """A capsule embedded in the solid outside a thin pipe has no fluid node
    in any support (no coupling), so its vertices follow the Verlet history
    alone: v0 = -3 (x - c) gives x^{-1} = x + 3 (x - c) and stretches every
    edge 2.5x in the first step, which must stop the computation there."""
    d = synth.pipe(24, 24, 24, 3.0, periodic_x=True, init="rest")
    X, Fc = synth.icosphere(2, 3.0, (12.0, 4.0, 4.0))
    v0 = -3.0 * (X - np.array([12.0, 4.0, 4.0]))
    b = synth.Body(X, Fc, rigid=False, ca=0.05, r_ref=3.0, u_ref=0.02, v0=v0)
    s = oracle.OracleSim(d, tau=0.8, u_max=0.02, bodies=[b], threads=2)
    assert s.step(3) == 5  # damaged
    assert s.steps_done == 1
    x1, _ = s.body(0)
    assert np.abs(x1 - (X + 1.5 * (X - [12.0, 4.0, 4.0]))).max() < 1e-12
    assert s.step(1) == 5 and s.steps_done == 1
    assert np.array_equal(s.body(0)[0], x1)


def test_unstable_flow_is_flagged():
    d = synth.periodic_box(8, 8, 8)
    d.init_u = np.full(3 * d.n_nodes, 0.4)
    s = oracle.OracleSim(d, tau=0.8, threads=1)
    assert s.step(2) == 4 and s.steps_done == 1


# -------------------------------------------- BFL second-order wall convergence
def _channel_error(nz, q0, tau, g=1e-6, relax=2.0):
    """Body-force-driven plane Poiseuille flow between flat walls crossing
    every wall link at fraction q0 (walls at z = 1 - q0 and nz - 2 + q0),
    periodic in x and y.  Returns max |u - u_exact| / u_max at steady state."""
    nx = ny = 2
    N = nx * ny * nz
    i = np.arange(N)
    z = i // (nx * ny)
    nt = np.where((z == 0) | (z == nz - 1), 1, 0).astype(np.uint8)
    E = synth.D3Q19_DIRS
    ln, ld = [], []
    for n in i[(z == 1) | (z == nz - 2)]:
        for k in range(1, 19):
            if (z[n] == 1 and E[k, 2] == -1) or (z[n] == nz - 2 and E[k, 2] == 1):
                ln.append(n)
                ld.append(k)
    d = synth.Domain(nx, ny, nz, (True, True, False), nt, np.array(ln, np.int64),
                     np.array(ld, np.uint8), np.full(len(ln), q0), np.zeros(0), 1.0,
                     None, None, (g, 0.0, 0.0))
    s = oracle.OracleSim(d, tau=tau, threads=1)
    nu = (tau - 0.5) / 3
    H = (nz - 3) + 2 * q0
    s.step(int(relax * H * H / nu))
    _, u = s.fields()
    z0, z1 = 1 - q0, nz - 2 + q0
    zz = z[nt == 0]
    ua = g / (2 * nu) * (zz - z0) * (z1 - zz)
    return np.abs(u[0][nt == 0] - ua).max() / ua.max()


def test_halfway_bounce_back_exact_at_magic_tau():
    """With q = 1/2 the rule is the halfway bounce-back, which for BGK
    reproduces plane Poiseuille flow exactly when (tau - 1/2)^2 = 3/16."""
    assert _channel_error(12, 0.5, 0.5 + np.sqrt(3) / 4, relax=5.0) < 1e-9


@pytest.mark.parametrize("q0", [0.25, 0.75])
def test_bfl_second_order_wall_convergence(q0):
    errs = np.array([_channel_error(nz, q0, 0.8) for nz in (12, 22, 42)])
    H = np.array([9, 19, 39]) + 2 * q0
    slope = -np.polyfit(np.log(H), np.log(errs), 1)[0]
    assert slope > 1.8, (errs, slope)


def _poiseuille_error(R, tau=1.0, g=1e-6):
    n = int(2 * np.ceil(R) + 4)
    d = synth.pipe(2, n, n, R, periodic_x=True, init="rest", body_force=(g, 0, 0))
    s = oracle.OracleSim(d, tau=tau, threads=2)
    nu = (tau - 0.5) / 3
    s.step(int(8 * R * R / nu))
    rho, u = s.fields()
    i = np.arange(d.n_nodes)
    y, z = (i // 2) % n, i // (2 * n)
    r2 = (y - (n - 1) / 2) ** 2 + (z - (n - 1) / 2) ** 2
    fl = d.node_type != 1
    ua = g * (R * R - r2) / (4 * nu)
    return np.sqrt(np.sum((u[0][fl] - ua[fl]) ** 2) / np.sum(ua[fl] ** 2))


def test_pipe_poiseuille_profile():
    """Hagen-Poiseuille flow in the circular pipe with the interpolated
    walls: L2 error below 1% at R = 8 and decreasing with R."""
    e8, e12 = _poiseuille_error(8.0), _poiseuille_error(12.0)
    assert e8 < 0.01 and e12 < e8


def test_bfl_second_order_on_a_curved_wall():
    """The interpolated bounce-back on the curved wall of a circular pipe
    (radii off the lattice, so the link fractions vary around the wall):
    the L2 error of Hagen-Poiseuille flow falls as R^-2 (fitted slope over
    R = 4.3, 8.3, 16.3 above 1.6; measured 2.0)."""
    R = np.array([4.3, 8.3, 16.3])
    errs = np.array([_poiseuille_error(r) for r in R])
    slope = -np.polyfit(np.log(R), np.log(errs), 1)[0]
    assert slope > 1.6, (errs, slope)


def test_stokes_drag_on_a_fixed_sphere():
    """A fixed rigid sphere (radius 3, 162 vertices) in a periodic 24^3 box
    of fluid driven by a uniform body force g at low Reynolds number.  At the
    steady state the immersed-boundary force spread on the fluid balances
    the body force exactly (sum f_ib = -g N), and the drag F = g N against
    the mean velocity U follows Stokes' law for a periodic array of spheres
    (Hasimoto's correction K(phi) to 6 pi mu R U).  The diffuse interface
    makes the sphere act slightly larger than R: F / (6 pi mu R U K) is 1.07
    here; it is held to [0.95, 1.15]."""
    L, R, tau, g = 24, 3.0, 1.0, 1e-6
    d = synth.periodic_box(L, L, L, body_force=(g, 0.0, 0.0))
    X, F = synth.icosphere(2, R, (11.7, 11.6, 11.55), tilt=True)
    b = synth.Body(X, F, rigid=True, fixed=True, rho_ratio=1.1, r_ref=R)
    s = oracle.OracleSim(d, tau=tau, u_max=0.0, bodies=[b], threads=4)
    assert s.step(9000) == 0
    _, u = s.fields()
    fib = s.force()
    N = L ** 3
    np.testing.assert_allclose(fib.sum(1), [-g * N, 0.0, 0.0], rtol=2e-4, atol=2e-4 * g * N)
    nu = (tau - 0.5) / 3.0
    U = u[0].mean()
    phi = 4.0 / 3.0 * np.pi * R ** 3 / N
    K = 1.0 / (1.0 - 1.7601 * phi ** (1 / 3) + phi - 1.5593 * phi ** 2)
    ratio = g * N / (6.0 * np.pi * nu * R * U * K)
    assert 0.95 < ratio < 1.15, ratio


# ------------------------------------------------- repulsion (Eq. collision)

@pytest.mark.parametrize("d", [0.3, 0.55, 0.9])
def test_repulsion_closed_form_for_one_facing_pair(d):
    """Fluid at rest around two fixed bodies: the hydrodynamic force
    vanishes, and the external force is the repulsion alone.  Only the
    facing pair is within one spacing, so each facing face is pushed along
    its inward normal (away from the other body) with magnitude
    u_max/(8 sqrt 2) d^(-5/2); every other face feels nothing."""
    w = synth.facing_pair(d)
    u_max, f0 = w.u_max, w.meta["face"]
    s = oracle.OracleSim(w.domain, tau=w.tau, u_max=u_max, bodies=w.bodies, threads=1)
    assert s.step(1) == 0
    mag = u_max / (8.0 * np.sqrt(2.0)) * d ** -2.5
    for bid, sign in ((0, -1.0), (1, 1.0)):
        Fe = s.body_fext(bid)
        np.testing.assert_allclose(Fe[f0], [sign * mag, 0.0, 0.0], rtol=1e-12, atol=1e-13)
        rest = np.delete(Fe, f0, axis=0)
        assert np.abs(rest).max() < 1e-13
    # Newton's third law for the pair
    np.testing.assert_allclose(s.body_fext(0).sum(0), -s.body_fext(1).sum(0), atol=1e-13)


def test_repulsion_vanishes_beyond_one_spacing():
    w = synth.facing_pair(1.05)
    s = oracle.OracleSim(w.domain, tau=w.tau, u_max=w.u_max, bodies=w.bodies, threads=1)
    assert s.step(1) == 0
    assert np.abs(s.body_fext(0)).max() < 1e-13 and np.abs(s.body_fext(1)).max() < 1e-13


# ------------------------------------------------ property tests (hypothesis)
from hypothesis import given, settings, strategies as st  # noqa: E402

_finite = dict(allow_nan=False, allow_infinity=False)


@settings(max_examples=40, deadline=None)
@given(r=st.floats(0.0, 4.4, **_finite), t=st.floats(0.0, 6.283, **_finite),
       xp=st.floats(0.0, 11.0, **_finite), a=st.floats(-2.0, 2.0, **_finite),
       g=st.tuples(*[st.floats(-1.0, 1.0, **_finite)] * 3))
def test_mls_reproduces_linear_fields_anywhere(r, t, xp, a, g):
    """Any point of the pipe, any linear field: the MLS weights reproduce its
    value and gradient (also where the support is cut by the wall)."""
    d, s = _pipe_sim()
    p = np.array([xp, 5.5 + r * np.cos(t), 5.5 + r * np.sin(t)])
    ok, node, psi = s.mls_point(p)
    assert ok
    G = np.array(g)
    x = np.stack([node % 12, (node // 12) % 12, node // 144], 1).astype(float)
    x[:, 0] += 12 * np.round((p[0] - x[:, 0]) / 12)
    m = node >= 0
    val = a + (x[m] - p) @ G
    assert abs(psi[m, 0] @ val - a) < 1e-11
    assert np.abs(psi[m, 1:].T @ val - G).max() < 1e-11


@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 2 ** 31 - 1), amp=st.floats(0.01, 0.3, **_finite),
       which=st.sampled_from([1, 2, 4, 7]))
def test_membrane_balance_on_random_shapes(seed, amp, which):
    """Randomly deformed capsules: stretching, bending and volume forces
    (and their sum) exert no net force or torque."""
    b, s = _capsule_sim()
    x = b.x + np.random.default_rng(seed).normal(scale=amp, size=b.x.shape)
    _, F = s.membrane(0, x, which)
    scale = max(np.abs(F).max(), 1e-300)
    assert np.abs(F.sum(0)).max() < 1e-12 * scale * len(x)
    assert np.abs(np.cross(x, F).sum(0)).max() < 1e-11 * scale * len(x)


def test_set_populations_is_the_inverse_of_get():
    """Handing one simulation's populations to another makes it step on as
    the first does (the state is the post-collision populations alone)."""
    w = synth.tiny_pipe(with_body=False)
    a = oracle.from_workload(w, threads=1)
    a.step(4)
    b = oracle.OracleSim(synth.pipe(24, 12, 12, 4.5, u_max=0.05, tau=0.8, init="rest"), 0.8, 0.05, threads=1)
    b.set_populations(a.populations())
    assert np.abs(b.populations() - a.populations()).max() <= 1e-16
    a.step(5)
    b.step(5)
    assert np.abs(b.populations() - a.populations()).max() <= 1e-15


# ------------------------------------------------ rigid-body rotation (S8)
def _box_mesh(a, b, c, center, Q=np.eye(3)):
    """Closed triangle mesh of an a x b x c box (8 corners, 12 faces, outward
    counter-clockwise), its edges along the columns of the rotation Q."""
    corners = np.array([[(i - 0.5) * a, (j - 0.5) * b, (k - 0.5) * c]
                        for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    quads = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]
    tris = []
    for q in quads:
        for t in ((q[0], q[1], q[2]), (q[0], q[2], q[3])):
            p = corners[list(t)]
            if np.dot(np.cross(p[1] - p[0], p[2] - p[0]), p.mean(0)) < 0:
                t = (t[0], t[2], t[1])
            tris.append(t)
    return corners @ Q.T + np.asarray(center), np.array(tris, dtype=np.int32)


def _rot(axis, angle):
    from scipy.spatial.transform import Rotation
    axis = np.asarray(axis, float)
    return Rotation.from_rotvec(angle * axis / np.linalg.norm(axis)).as_matrix()


def _rigid_sim(X, F, rho_ratio=1.3):
    d = synth.periodic_box(24, 24, 24)
    body = synth.Body(X, F, rigid=True, ca=0.05, eb=0.0, rho_ratio=rho_ratio, r_ref=2.0, u_ref=0.02)
    return oracle.OracleSim(d, tau=0.8, u_max=0.02, bodies=[body], threads=1)


@pytest.mark.parametrize("rotated", [False, True])
def test_rigid_inertia_exact_on_box_meshes(rotated):
    """The inertia of the uniform solid inside a closed box mesh is the
    textbook m (b^2 + c^2) / 12 etc. along its edges, whatever its position
    and orientation.  The box sits away from the origin and is anisotropic:
    a missing shift to the centre of mass, the second-moment matrix C used
    in place of tr(C) 1 - C, a wrong 1/20 tetrahedron factor or a sign error
    in the products of inertia (the rotated case) each fail."""
    a, b, c, rr = 3.0, 2.0, 1.2, 1.3
    Q = _rot((0.3, -0.5, 0.8), 0.9) if rotated else np.eye(3)
    X, F = _box_mesh(a, b, c, (10.3, 11.7, 12.2), Q)
    s = _rigid_sim(X, F, rr)
    m = rr * a * b * c
    assert abs(s.body_diag(0)["mass"] - m) < 1e-12 * m
    I_ref = Q @ np.diag([m * (b * b + c * c) / 12, m * (a * a + c * c) / 12, m * (a * a + b * b) / 12]) @ Q.T
    assert np.abs(s.body_inertia(0) - I_ref).max() < 1e-12 * np.abs(I_ref).max()
    assert np.abs(s.body_diag(0)["xc"] - [10.3, 11.7, 12.2]).max() < 1e-12


def test_rigid_inertia_of_refined_icospheres_tends_to_the_solid_sphere():
    """For icospheres of radius r the mesh inertia is isotropic and I / (m r^2)
    approaches the solid sphere's 2/5 as the mesh is refined, with the error
    shrinking about four times per subdivision (second order in the edge)."""
    r = 5.0
    errs = []
    for sub in range(1, 5):
        X, F = synth.icosphere(sub, r, (11.1, 12.3, 11.6), tilt=True)
        s = _rigid_sim(X, F)
        I = s.body_inertia(0)
        m = s.body_diag(0)["mass"]
        assert np.abs(I - np.diag(np.diag(I))).max() < 1e-12 * I[0, 0]
        assert np.ptp(np.diag(I)) < 1e-3 * I[0, 0] / 4 ** sub
        errs.append(abs(I[0, 0] / (m * r * r) - 0.4))
    assert errs[-1] < 2e-3
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.0 < e0 / e1 < 5.0


def test_rodrigues_matches_scipy():
    """The oracle's rotation matrix of a rotation vector equals scipy's
    (a transposed matrix, a sign error in the cross-product term or a wrong
    1 - cos term would each fail), including tiny and large angles."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(7)
    vecs = [rng.normal(size=3) * s for s in (1e-9, 1e-4, 0.05, 0.7, 2.0, 3.1)]
    vecs += [np.array([np.pi, 0, 0]), np.array([0.0, 0.0, 0.0])]
    for phi in vecs:
        R = oracle.rodrigues(phi)
        assert np.abs(R - Rotation.from_rotvec(phi).as_matrix()).max() < 2e-15
        assert np.abs(R @ R.T - np.eye(3)).max() < 2e-15 and np.linalg.det(R) > 0


@pytest.mark.parametrize("rotated", [False, True])
def test_rigid_second_order_backward_recurrence(rotated):
    """Constant force f on every corner and a torque about a principal axis e
    (corner forces s e x (x_v - x_c), the same moment at every step) drive a
    box from rest.  The second-order backward update
    u^{n+1} = 2/3 (2 u^n - u^{n-1}/2 + F/m) from u^0 = u^{-1} = 0 has the
    closed form u^n = (F/m)(n - 1/2 + 3^{-n}/2), and likewise omega^n with
    M/I_e; the centre moves by the sum of the u^k and the body turns about e
    by the sum of the |omega^k| (rotations about one axis commute).  A sign
    slip in the angular update, a transposed rotation (turning the wrong
    way), a wrong inertia or wrong history weights each fail."""
    a, b, c, rr = 3.0, 2.0, 1.2, 1.3
    Q = _rot((0.3, -0.5, 0.8), 0.9) if rotated else np.eye(3)
    c0 = np.array([10.3, 11.7, 12.2])
    X, F = _box_mesh(a, b, c, c0, Q)
    s = _rigid_sim(X, F, rr)
    m = rr * a * b * c
    e = Q[:, 2]                               # principal axis of I_e = m (a^2 + b^2) / 12
    I_e = m * (a * a + b * b) / 12
    f = np.array([2e-4, -1e-4, 3e-4])
    sm = 3e-4
    M = sm * 2 * (a * a + b * b)              # sum over corners of r x (e x r) along e
    xc_ref = c0.copy()
    theta = 0.0
    for n in range(1, 13):
        x, _ = s.body(0)
        xc = s.body_diag(0)["xc"]
        Fv = f + sm * np.cross(e, x - xc)
        assert s.move_rigid(0, Fv) == 0
        k = n - 0.5 + 0.5 * 3.0 ** (-n)
        u_ref = 8 * f / m * k
        w_ref = M / I_e * k * e
        dg = s.body_diag(0)
        assert np.abs(dg["u"] - u_ref).max() < 1e-12 * np.abs(u_ref).max()
        assert np.abs(dg["omega"] - w_ref).max() < 1e-12 * np.abs(w_ref).max()
        xc_ref += u_ref
        theta += np.linalg.norm(w_ref)
        assert np.abs(dg["xc"] - xc_ref).max() < 1e-12
        x, v = s.body(0)
        x_ref = xc_ref + (X - c0) @ _rot(e, theta).T
        assert np.abs(x - x_ref).max() < 1e-12
        # vertex velocities are the rigid motion's
        assert np.abs(v - (u_ref + np.cross(w_ref, x - xc_ref))).max() < 1e-13
    assert theta > 0.05                       # the box really turned


def test_rigid_rotations_compose_in_the_world_frame():
    """A cube (isotropic inertia m a^2 / 6 in any orientation) driven by
    moments about changing axes: each step's rotation Rodrigues(omega^{n+1})
    acts in the world frame after the previous ones, R <- R(omega) R.  The
    reference composes scipy rotations in that order; composing in the body
    frame (R R(omega)) or transposing either factor fails, since rotations
    about different axes do not commute."""
    from scipy.spatial.transform import Rotation
    a, rr = 2.5, 1.2
    c0 = np.array([11.2, 12.4, 11.8])
    X, F = _box_mesh(a, a, a, c0, _rot((1.0, 2.0, -0.5), 0.4))
    s = _rigid_sim(X, F, rr)
    m = rr * a ** 3
    I = m * a * a / 6
    axes = [np.array(v, float) / np.linalg.norm(v) for v in
            ((1, 0, 0), (1, 0, 0), (0, 1, 0), (0, 1, 0), (0, 0.6, 0.8), (1, 1, 0), (0, 0, 1), (1, -1, 1))]
    sm = 5e-3
    w, wprev = np.zeros(3), np.zeros(3)
    R = Rotation.identity()
    for d in axes:
        x, _ = s.body(0)
        xc = s.body_diag(0)["xc"]
        assert s.move_rigid(0, sm * np.cross(d, x - xc)) == 0
        M = 4 * sm * a * a * d                # sum over corners of r x (d x r)
        w, wprev = 2.0 / 3.0 * (2 * w - 0.5 * wprev + M / I), w
        R = Rotation.from_rotvec(w) * R       # world-frame increment after the previous ones
        dg = s.body_diag(0)
        assert np.abs(dg["omega"] - w).max() < 1e-12 * np.abs(w).max()
        x, _ = s.body(0)
        assert np.abs(x - (c0 + (X - c0) @ R.as_matrix().T)).max() < 1e-12
    assert R.magnitude() > 0.1


# ------------------------------------------ storage form of the populations
_STORAGE_RUN = '''
import sys
import numpy as np
sys.path.insert(0, {root!r})
import oracle, synth
if sys.argv[1]:
    oracle.use_library(sys.argv[1])
w = synth.tiny_bifurcation(precision="f64", n_bodies=0)
s = oracle.from_workload(w, with_bodies=False, threads=2)
assert s.step(600) == 0
np.save(sys.argv[2], s.fields()[1])
'''


def test_deviation_storage_is_nearer_the_exact_trajectory(tmp_path):
    """The oracle stores populations as deviations f - w; storing full
    populations instead is the same map in exact arithmetic.  Against a
    long-double run of the same source (rounding ~2^-64) on a small
    bifurcation after 600 steps, the double oracle stays within 3e-14 of the
    velocity scale, while full-population storage drifts more than ten times
    further: its rounding of values near w_i has the same sign step after
    step.  (The full-size workload: tests/golden/storage_form.json, written by
    make_storage_form.py: 1.3e-14 against 1.1e-12 after 2000 steps.)"""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "run.py"
    script.write_text(_STORAGE_RUN.format(root=root))
    res = {}
    for b in ("ldouble", "fullpop", "plain"):
        lib = "" if b == "plain" else oracle.build(variant=b, path=str(tmp_path / f"{b}.so"))
        subprocess.run([sys.executable, str(script), lib, str(tmp_path / f"{b}.npy")], check=True)
        res[b] = np.load(tmp_path / f"{b}.npy")
    fl = synth.tiny_bifurcation(precision="f64", n_bodies=0).domain.node_type != synth.SOLID
    ref = res["ldouble"][:, fl]
    e = {b: np.abs(res[b][:, fl] - ref).max() / np.abs(ref).max() for b in ("plain", "fullpop")}
    assert e["plain"] < 3e-14, e
    assert e["fullpop"] > 10 * e["plain"], e
