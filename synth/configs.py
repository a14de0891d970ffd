"""Named synthetic workloads.

Each generator returns a :class:`Workload`: a lattice domain, the bodies to
release in it, the relaxation time, the characteristic velocity u_max (used
by the inter-body repulsion), the population precision and the number of
steps.  Sizes and parameters follow the configurations the build is measured
on; random draws use ``numpy.random.default_rng(seed)`` in the documented
order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .geometry import D3Q19_DIRS, OUTLET, SOLID, Domain, bifurcation, periodic_box, pipe
from .mesh import Body, icosphere, off_switch_planes


@dataclass
class Workload:
    name: str
    domain: Domain
    bodies: list
    tau: float
    u_max: float
    precision: str          # "f64" | "f32" | "f16s"
    steps: int
    meta: dict = field(default_factory=dict)


def pipe_sphere(precision="f64", steps=200):
    """Straight pipe D = 16 on a 48x20x20 grid, tau = 0.8, Poiseuille inlet
    u_max = 0.05, outlet rho = 1, one rigid icosphere (subdivision 2, 162
    vertices, in the fixed tilted orientation) of radius 4 released at rest on
    the axis at x = 12, density ratio 1.1.  No random draws."""
    tau, u_max = 0.8, 0.05
    dom = pipe(48, 20, 20, 8.0, u_max=u_max, tau=tau, init="poiseuille")
    X, F = icosphere(2, 4.0, (12.0, 9.5, 9.5), tilt=True)
    assert off_switch_planes(X, F)
    body = Body(X, F, rigid=True, rho_ratio=1.1, r_ref=4.0, u_ref=u_max)
    return Workload("pipe_sphere", dom, [body], tau, u_max, precision, steps)


def bifurcation_capsule(seed=0, precision="f32", steps=5000, nx=256, ny=128, nz=40,
                        D=32.0, subdiv=4, occlusion=0.5, ca=0.01, eb=1e-4):
    """Symmetric Y-bifurcation, main diameter D = 32, daughters 0.8 D at a
    60 degree semi-aperture, fillet radius 4, grid 256x128x40, Re = 10 with
    tau = 0.7 (so u_max = Re*nu/D), one deformable icosphere capsule
    (subdivision 4, 2562 vertices) at occlusion ratio 0.5 with Ca = 0.01,
    density ratio 1.1, released at x = 1.16 D with a lateral offset drawn
    first from U[-0.1 D, 0.1 D].  The mesh is in the fixed tilted orientation
    so that no marker starts on the mid-plane z = (nz - 1)/2, a half-integer
    plane where the support of the 3x3x3 stencil would be chosen by rounding.

    Bending number: 1e-4 instead of the paper's 1e-3.  For this mesh (rest
    edge ~0.6 lu, vertex mass ~0.92) the largest bending mode of the rest
    shape has lambda/m_v = 0.88 at Eb = 1e-3, beyond the ~0.85 limit of the
    explicit vertex update, and the capsule is damaged after ~860 steps;
    at Eb = 1e-4 it is 0.09 (the stretching modes are at 0.78)."""
    rng = np.random.default_rng(seed)
    tau = 0.7
    nu = (tau - 0.5) / 3.0
    u_max = 10.0 * nu / D
    dom = bifurcation(nx, ny, nz, D, 0.8, 60.0, 4.0, u_max=u_max)
    rp = occlusion * D / 2.0
    dy = rng.uniform(-0.1 * D, 0.1 * D)
    c = (1.16 * D, (ny - 1) / 2.0 + dy, (nz - 1) / 2.0)
    X, F = icosphere(subdiv, rp, c, tilt=True)
    assert off_switch_planes(X, F)
    body = Body(X, F, rigid=False, ca=ca, eb=eb, rho_ratio=1.1, r_ref=rp, u_ref=u_max)
    return Workload("bifurcation_capsule", dom, [body], tau, u_max, precision, steps,
                    meta={"offset": dy, "seed": seed})


# Stability guard of the capsule stiffness.  The explicit vertex update
# (Verlet predictor, BDF2 velocity, corrector) diverges once the largest
# eigenvalue of the membrane stiffness over the vertex mass passes about
# 0.8 (the 2562-vertex capsule of the Y-bifurcation is stable at 0.75 and
# fails at 0.85).  The largest stretching eigenvalue of the icosphere spring
# network at rest is 5.2 k_s0 for every subdivision used here, so a capsule
# is only given a capillary number for which 5.2 k_s0 / m_v <= 0.6.
STRETCH_EIG = 5.2
STIFFNESS_LIMIT = 0.6


def _mesh_volume(X, F):
    a, b, c = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def ca_floor(X, F, nu, u_ref, rho_ratio):
    """Smallest capillary number Ca = nu u_ref / k_s0 (fluid density 1) that
    keeps 5.2 k_s0 / m_v <= 0.6, with m_v = rho_ratio V / n_v the vertex
    mass of the mesh (X, F)."""
    m_v = rho_ratio * _mesh_volume(X, F) / len(X)
    return nu * u_ref / (STIFFNESS_LIMIT * m_v / STRETCH_EIG)


# Unit directions at which the wall clearance of a capsule candidate is
# checked (icosphere vertices, 642 directions, about 8 degrees apart).
_CLEAR_DIRS = None


def _clear_of_walls(sdf, c, radius):
    """True when the sphere of the given radius around c lies in the fluid:
    the signed distance is negative at its centre and at 642 points of its
    surface.  (The smooth union of the tubes keeps the sign of the signed
    distance exact but overstates the depth where two tubes overlap, so the
    depth at the centre alone is not a clearance test.)"""
    global _CLEAR_DIRS
    if _CLEAR_DIRS is None:
        _CLEAR_DIRS = icosphere(3, 1.0)[0]
    pts = np.vstack([c[None, :], c[None, :] + radius * _CLEAR_DIRS])
    return bool(np.all(sdf(pts) < 0.0))


def _place_capsules(rng, sdf, box, D, n, occl_lo, occl_hi, ca_lo, ca_hi, subdiv_choices,
                    x_inlet_clear, face_clear, u_max, nu, eb=1e-4, max_tries=100000,
                    tries_per_capsule=2000, x_max=None):
    """Rejection sampling of non-overlapping capsules inside the fluid.
    Draw order per capsule: occlusion ratio, mesh choice, log10 Ca uniform
    on [log10 max(ca_lo, ca_floor), log10 ca_hi] (ca_floor: the stability
    guard above; a capsule whose floor exceeds ca_hi is drawn again), then
    centre candidates (x, y, z) until one fits: the sphere of radius r_p + 1.5
    in the fluid (``_clear_of_walls``), centre distance >= r_i + r_j + 2 to
    the capsules already placed, at least x_inlet_clear from the inlet and
    face_clear from the other faces, and x <= x_max if given.  A capsule that finds no centre within
    tries_per_capsule candidates is drawn again (occlusion, mesh, Ca) from
    the same stream; the redraws are counted.  Returns (bodies, redraws);
    stops early once max_tries candidates have been spent."""
    nx, ny, nz = box
    bodies, centres, radii = [], [], []
    tries = redraws = 0
    while len(bodies) < n and tries < max_tries:
        occ = rng.uniform(occl_lo, occl_hi)
        sub = subdiv_choices[rng.integers(len(subdiv_choices))]
        rp = occ * D / 2.0
        Xu, Fu = icosphere(sub, rp, (0.0, 0.0, 0.0), tilt=True)
        lo = max(ca_lo, ca_floor(Xu, Fu, nu, u_max, 1.1))
        if lo > ca_hi:
            redraws += 1
            continue
        ca = 10.0 ** rng.uniform(np.log10(lo), np.log10(ca_hi))
        placed = None
        for _ in range(tries_per_capsule):
            if tries >= max_tries:
                break
            tries += 1
            x_hi = nx - 1 - face_clear if x_max is None else min(nx - 1 - face_clear, x_max)
            c = np.array([rng.uniform(x_inlet_clear, x_hi),
                          rng.uniform(face_clear, ny - 1 - face_clear),
                          rng.uniform(0, nz - 1)])
            if sdf(c[None, :])[0] > -(rp + 1.5) or not _clear_of_walls(sdf, c, rp + 1.5):
                continue
            if any(np.linalg.norm(c - cc) < rp + rr + 2.0 for cc, rr in zip(centres, radii)):
                continue
            placed = c
            break
        if placed is None:
            redraws += 1
            continue
        X, F = Xu + placed, Fu
        if not off_switch_planes(X, F):
            redraws += 1
            continue
        bodies.append(Body(X, F, rigid=False, ca=ca, eb=eb, rho_ratio=1.1, r_ref=rp, u_ref=u_max))
        centres.append(placed)
        radii.append(rp)
    return bodies, redraws


def precision_form(seed=0, precision="f16s", steps=2000, n_capsules=16):
    """Bifurcation with a 90 degree semi-aperture on 512x256x64, D = 48,
    fillet 4, Re = 10 with tau = 0.7, 16 deformable capsules (2562 vertices)
    with occlusion ratio ~ U[0.3, 0.8] and Ca log-uniform in [1e-3, 1e-1]
    above the stability floor ``ca_floor`` (which only binds for the smaller
    capsules), Eb = 1e-4 as for the single capsule, placed without overlap at
    least 1 D from the inlet and the outlet faces."""
    rng = np.random.default_rng(seed)
    tau = 0.7
    nu = (tau - 0.5) / 3.0
    D = 48.0
    u_max = 10.0 * nu / D
    dom = bifurcation(512, 256, 64, D, 0.8, 90.0, 4.0, u_max=u_max)
    bodies, redraws = _place_capsules(rng, dom.meta["sdf"], (512, 256, 64), D, n_capsules,
                                      0.3, 0.8, 1e-3, 1e-1, (4,), D, D, u_max, nu)
    return Workload("precision_form", dom, bodies, tau, u_max, precision, steps,
                    meta={"seed": seed, "radius_redraws": redraws})


def batch_instance(seed, k):
    """Instance k of the batching form: the draws come from its own stream
    numpy.random.default_rng([seed, k]), in the order D from {16, 24, 32,
    48}, semi-aperture U[30, 120] degrees, fillet U[0, 0.25 D], the number of
    capsules (1-4), then the capsules (occlusion U[0.3, 0.9], 642 or 2562
    vertices, Ca log-uniform in [1e-3, 1e-1] above the stability floor
    ``ca_floor``, Eb = 1e-4) on an 8D x 4D x 1.25D grid, Re = 10, tau = 0.7.
    Capsule centres lie between 1 D after the inlet and 1.5 D before the
    junction (x <= 2.5 D): at D = 16 the capsules travel about 1.3 D in the
    1000 steps, so none reaches the junction apex, where capsules are
    stretched until the damage stop, or an outlet (the method has no
    treatment of a capsule crossing an open face).  The nodes on the box
    edges are solid (a daughter tube at a small angle leaves through the
    edge x = nx - 1, y = 0 or ny - 1)."""
    rng = np.random.default_rng([seed, k])
    D = float(rng.choice([16, 24, 32, 48]))
    th = rng.uniform(30.0, 120.0)
    fil = rng.uniform(0.0, 0.25 * D)
    ncap = int(rng.integers(1, 5))
    nx, ny, nz = int(8 * D), int(4 * D), int(1.25 * D)
    tau = 0.7
    nu = (tau - 0.5) / 3.0
    u_max = 10.0 * nu / D
    dom = bifurcation(nx, ny, nz, D, 0.8, th, fil, x_junction=4 * D, u_max=u_max,
                      edge_band=0.5)
    bodies, redraws = _place_capsules(rng, dom.meta["sdf"], (nx, ny, nz), D, ncap, 0.3, 0.9,
                                      1e-3, 1e-1, (3, 4), D, D, u_max, nu, x_max=2.5 * D)
    return Workload(f"batch_{k}", dom, bodies, tau, u_max, "f32", 1000,
                    meta={"D": D, "theta": th, "fillet": fil, "seed": seed, "index": k,
                          "radius_redraws": redraws})


def _batch_instance_no_sdf(seed, k):
    w = batch_instance(seed, k)
    w.domain.meta["sdf"] = None  # a closure: not sent between processes
    return w


def batch_instances(seed=0, n_instances=64, workers=1):
    """The batching form: instances 0 .. n_instances-1 of ``batch_instance``
    (each from its own random stream, so any prefix is the same and the
    instances can be generated in parallel by ``workers`` processes; those
    come back without the signed-distance function in domain.meta)."""
    if workers <= 1:
        return [batch_instance(seed, k) for k in range(n_instances)]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_batch_instance_no_sdf, [seed] * n_instances, range(n_instances)))


def periodic_r0(n=256, precision="f32", steps=100):
    """All-fluid periodic n^3 box driven by a uniform body force 1e-6 along
    x, tau = 0.8 (the stream-collide bandwidth ceiling workload)."""
    dom = periodic_box(n, n, n, body_force=(1e-6, 0.0, 0.0))
    return Workload(f"periodic_{n}", dom, [], 0.8, 0.0, precision, steps)


def pipe_r1(precision="f32", steps=100):
    """Straight pipe D = 96 in a 768x100x100 box, Poiseuille inlet u_max =
    0.05, outlet rho = 1, tau = 0.8 (walls + open faces at scale)."""
    dom = pipe(768, 100, 100, 48.0, u_max=0.05, tau=0.8, init="poiseuille")
    return Workload("pipe_r1", dom, [], 0.8, 0.05, precision, steps)


def tiny_pipe(precision="f64", steps=20, with_body=True, rigid=True, nx=24, ny=12, nz=12,
              radius=4.5, body_radius=2.5, subdiv=2):
    """Small pipe for quick parity checks (several tiles, ragged rows)."""
    tau, u_max = 0.8, 0.05
    dom = pipe(nx, ny, nz, radius, u_max=u_max, tau=tau, init="poiseuille")
    bodies = []
    if with_body:
        X, F = icosphere(subdiv, body_radius, (7.3, (ny - 1) / 2.0 + 0.21, (nz - 1) / 2.0 - 0.13))
        bodies.append(Body(X, F, rigid=rigid, ca=0.2, eb=0.001, rho_ratio=1.1,
                           r_ref=body_radius, u_ref=u_max))
    return Workload("tiny_pipe", dom, bodies, tau, u_max, precision, steps)


def facing_pair(d=0.5, subdiv=0, radius=3.0, rigid=True, fixed=True, precision="f64", steps=1,
                u_max=0.04, centre=(11.3, 7.9, 8.2), box=(24, 16, 16)):
    """Two icospheres in a periodic box of fluid at rest, mirror images of
    each other through the plane x = centre[0], with face 0 of each parallel
    to that plane and the two face-0 centroids a distance d apart on the
    x axis (the closest centroid pair of the two bodies).  No random draws.
    meta["face"] is the index of the facing face in both bodies."""
    X, F = icosphere(subdiv, 1.0)
    a, b, c = X[F[0, 0]], X[F[0, 1]], X[F[0, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n)
    # rotation taking the outward normal of face 0 onto +x (Rodrigues)
    ex = np.array([1.0, 0.0, 0.0])
    k = np.cross(n, ex)
    sn, cs = np.linalg.norm(k), float(n @ ex)
    k /= sn
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    R = np.eye(3) + sn * K + (1 - cs) * K @ K
    XA = (X @ R.T) * radius
    XA += np.asarray(centre) - XA[F[0]].mean(0) - np.array([d / 2, 0.0, 0.0])
    XB = XA.copy()
    XB[:, 0] = 2 * centre[0] - XB[:, 0]
    FB = F[:, [0, 2, 1]].copy()   # a mirror image reverses the orientation
    kw = dict(rigid=rigid, fixed=fixed and rigid, ca=0.05, eb=0.001, rho_ratio=1.1, r_ref=radius,
              u_ref=u_max)
    dom = periodic_box(*box)
    return Workload("facing_pair", dom, [Body(XA, F, **kw), Body(XB, FB, **kw)], 0.8, u_max,
                    precision, steps, meta={"face": 0, "d": d})


def tiny_bifurcation(seed=0, precision="f64", steps=20, n_bodies=1, subdiv=2):
    """Small Y-bifurcation (D = 12 on 64x40x16, 60 degrees, fillet 2) with
    one or two deformable capsules; draw order as in bifurcation_capsule."""
    rng = np.random.default_rng(seed)
    tau = 0.7
    nu = (tau - 0.5) / 3.0
    D = 12.0
    u_max = 0.02
    dom = bifurcation(64, 40, 16, D, 0.8, 60.0, 2.0, x_junction=32.0, u_max=u_max)
    bodies = []
    for k in range(n_bodies):
        dy = rng.uniform(-0.1 * D, 0.1 * D)
        rp = 2.6
        c = (10.0 + 5.4 * k, 19.5 + dy, 7.5 + (0.3 if k else 0.0))
        X, F = icosphere(subdiv, rp, c, tilt=True)
        assert off_switch_planes(X, F)
        bodies.append(Body(X, F, rigid=False, ca=0.05, eb=0.001, rho_ratio=1.1, r_ref=rp,
                           u_ref=u_max))
    del nu
    return Workload("tiny_bifurcation", dom, bodies, tau, u_max, precision, steps,
                    meta={"seed": seed})


TRAIN_KINDS = {"soft": ("soft", "soft", "soft"), "rigid_top": ("rigid", "soft", "soft"),
               "rigid_middle": ("soft", "rigid", "soft"), "rigid_bottom": ("soft", "soft", "rigid"),
               "all_rigid": ("rigid", "rigid", "rigid")}


def _train_bodies(kinds, x0, spacing, yc, zc, rp, ca, eb, u_ref, subdiv, rigid_subdiv):
    """A train along the axis: body k at x0 + k spacing (k = 0 the one
    nearest the inlet); "soft" a deformable capsule of radius rp, "rigid" a
    rigid sphere of half its diameter and the same density."""
    bodies = []
    for k, kind in enumerate(kinds):
        c = (x0 + k * spacing, yc, zc)
        if kind == "soft":
            X, F = icosphere(subdiv, rp, c, tilt=True)
            b = Body(X, F, rigid=False, ca=ca, eb=eb, rho_ratio=1.1, r_ref=rp, u_ref=u_ref)
        else:
            X, F = icosphere(rigid_subdiv, rp / 2.0, c, tilt=True)
            b = Body(X, F, rigid=True, ca=ca, eb=eb, rho_ratio=1.1, r_ref=rp / 2.0, u_ref=u_ref)
        assert off_switch_planes(X, F)
        bodies.append(b)
    return bodies


def capsule_train(train="soft", seed=0, precision="f32", steps=5000, theta_deg=60.0, junction="smooth",
                  ca=0.01, eb=1e-4):
    """A train of three capsules in the Y-bifurcation of the single-capsule
    workload (256x128x40, D = 32, daughters 0.8 D, fillet 4, Re = 10, tau =
    0.7) with the given junction ('smooth': the trapezoidal chamber with a
    flat wall; 'sharp').  Occlusion ratio 2/3 (r_p = D/3, 2562 vertices),
    the first capsule at 1.16 D from the inlet, the others downstream at a
    mutual centre distance of 0.85 D, all on the line y = (ny-1)/2 + dy with
    dy drawn first from U[-0.1 D, 0.1 D] (seed).  ``train`` picks the kinds
    (TRAIN_KINDS): all soft, one rigid sphere of half the capsule diameter
    in the top (nearest the inlet), middle or bottom place, or three rigid
    spheres.  Ca = 0.01 and Eb = 1e-4 (the bending number of the
    single-capsule workload)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz, D = 256, 128, 40, 32.0
    tau = 0.7
    nu = (tau - 0.5) / 3.0
    u_max = 10.0 * nu / D
    dom = bifurcation(nx, ny, nz, D, 0.8, theta_deg, 4.0, u_max=u_max, junction=junction)
    dy = rng.uniform(-0.1 * D, 0.1 * D)
    bodies = _train_bodies(TRAIN_KINDS[train], 1.16 * D, 0.85 * D, (ny - 1) / 2.0 + dy, (nz - 1) / 2.0,
                           D / 3.0, ca, eb, u_max, 4, 3)
    return Workload(f"capsule_train_{train}", dom, bodies, tau, u_max, precision, steps,
                    meta={"offset": dy, "seed": seed, "junction": junction, "train": train, "D": D})


def tiny_train(train="soft", seed=0, precision="f64", steps=30, junction="smooth"):
    """Small variant of capsule_train for parity checks: the 64x40x16
    bifurcation of tiny_bifurcation (D = 12) with the chosen junction and a
    train of three capsules of radius 2.6 (162 vertices) spaced 0.85 D from
    x = 6 (rigid: radius 1.3, 42 vertices)."""
    rng = np.random.default_rng(seed)
    tau, D, u_max = 0.7, 12.0, 0.02
    dom = bifurcation(64, 40, 16, D, 0.8, 60.0, 2.0, x_junction=32.0, u_max=u_max, junction=junction)
    dy = rng.uniform(-0.1 * D, 0.1 * D)
    bodies = _train_bodies(TRAIN_KINDS[train], 6.0, 0.85 * D, 19.5 + dy, 7.5, 2.6, 0.05, 0.001, u_max, 2, 1)
    return Workload(f"tiny_train_{train}", dom, bodies, tau, u_max, precision, steps,
                    meta={"seed": seed, "junction": junction, "train": train})


_REGISTRY = {
    "pipe_sphere": pipe_sphere,
    "bifurcation_capsule": bifurcation_capsule,
    "precision_form": precision_form,
    "periodic_r0": periodic_r0,
    "pipe_r1": pipe_r1,
    "tiny_pipe": tiny_pipe,
    "tiny_bifurcation": tiny_bifurcation,
    "facing_pair": facing_pair,
    "capsule_train": capsule_train,
    "tiny_train": tiny_train,
}


def outlet_flux_weights(domain):
    """Weights [19, N] of the outward fluxes of a bifurcation's two daughters:
    (w_up, w_lo), e_iy at the outlet nodes of the upper face (y = ny - 1) and
    -e_iy at those of the lower face (y = 0), zero elsewhere, so that
    <w, f> = <w, f - w_i> is the daughter's outward y-momentum flux."""
    ey = np.asarray(D3Q19_DIRS, dtype=np.float64)[:, 1]
    out = np.flatnonzero(domain.node_type == OUTLET)
    y = (out // domain.nx) % domain.ny
    w_up = np.zeros((19, domain.n_nodes))
    w_lo = np.zeros((19, domain.n_nodes))
    w_up[:, out[y == domain.ny - 1]] = ey[:, None]
    w_lo[:, out[y == 0]] = -ey[:, None]
    return w_up, w_lo


def terminal_weights(domain, seed):
    """Seeded weights [19, N]: one draw rng.normal(size=(19, N)) of
    default_rng(seed), zeroed at the solid nodes."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(19, domain.n_nodes)) * (domain.node_type != SOLID)


def get(name, **kw):
    return _REGISTRY[name](**kw)
