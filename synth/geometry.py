"""Lattice geometry generators: node tags, wall links and boundary data.

Conventions (shared interface with both solvers):

* Node (x, y, z) sits at lattice position (x, y, z); the linear index is
  ``x + nx*(y + ny*z)`` (x fastest).
* Node tags: ``FLUID`` 0, ``SOLID`` 1, ``INLET`` 2 (velocity Dirichlet),
  ``OUTLET`` 3 (density Dirichlet).  Inlet/outlet nodes are fluid nodes that
  sit on a non-periodic face of the box.
* A wall link ``(node, i, q)`` says that ``node + e_i`` is a solid node and
  that the wall crosses the segment from ``node`` to ``node + e_i`` at the
  fraction ``q`` of its length (the ratio defined next to the interpolated
  bounce-back rule in the section on stationary immersed boundaries).  ``i``
  indexes the D3Q19 velocity set in the order the paper prints it in the
  fluid-evolution section.
* Solid = outside the analytic fluid region (signed distance >= 0); the wall
  position along a link is the exact crossing for the straight pipe and a
  bisection to ~1e-16 on the signed distance for the bifurcation.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3

# Neighbour offsets in the order of the D3Q19 table printed in the paper's
# fluid-evolution section (columns 0..18 of the velocity matrix).  Only used
# here to enumerate neighbours when tagging wall links.
D3Q19_DIRS = np.array(
    [[0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0],
     [0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1],
     [0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1]],
    dtype=np.int64).T.copy()


@dataclass
class Domain:
    """A lattice domain ready to hand to either solver."""
    nx: int
    ny: int
    nz: int
    periodic: tuple
    node_type: np.ndarray            # uint8 [N]
    link_node: np.ndarray            # int64 [L]
    link_dir: np.ndarray             # uint8 [L]
    link_q: np.ndarray               # float64 [L]
    inlet_u: np.ndarray              # float64 [n_inlet*3], inlet nodes in index order
    outlet_rho: float = 1.0
    init_rho: np.ndarray | None = None   # float64 [N]
    init_u: np.ndarray | None = None     # float64 [3*N], component-major
    body_force: tuple = (0.0, 0.0, 0.0)
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.node_type != SOLID))

    def grid(self, a):
        """View a per-node array as [nz, ny, nx]."""
        return np.asarray(a).reshape(self.nz, self.ny, self.nx)


def _coords(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel().astype(np.float64), y.ravel().astype(np.float64), z.ravel().astype(np.float64)


def _tag_faces(nx, ny, nz, periodic, solid, inlet_faces):
    """Fluid nodes on non-periodic faces become INLET (faces listed in
    ``inlet_faces``) or OUTLET (all other faces).  A fluid node on two
    non-periodic faces is rejected."""
    nt = np.where(solid, SOLID, FLUID).astype(np.uint8).reshape(nz, ny, nx)
    count = np.zeros((nz, ny, nx), np.int32)
    faces = {0: (slice(None), slice(None), 0), 1: (slice(None), slice(None), nx - 1),
             2: (slice(None), 0, slice(None)), 3: (slice(None), ny - 1, slice(None)),
             4: (0, slice(None), slice(None)), 5: (nz - 1, slice(None), slice(None))}
    for f, sl in faces.items():
        if periodic[f // 2]:
            continue
        count[sl] += 1
    fluid = nt == FLUID
    if np.any(fluid & (count > 1)):
        raise ValueError("fluid node on a box edge/corner: the geometry must keep those solid")
    for f, sl in faces.items():
        if periodic[f // 2]:
            continue
        sub = nt[sl]
        sub[sub == FLUID] = INLET if f in inlet_faces else OUTLET
        nt[sl] = sub
    return nt.ravel()


def _links(nx, ny, nz, periodic, solid, qfun):
    """Enumerate (fluid node, direction) pairs whose neighbour is solid and
    attach q from ``qfun(points, dirs)``."""
    x, y, z = _coords(nx, ny, nz)
    idx = np.arange(nx * ny * nz, dtype=np.int64)
    nodes, dirs = [], []
    fluid = ~solid
    for i in range(1, 19):
        ex, ey, ez = D3Q19_DIRS[i]
        xn, yn, zn = x + ex, y + ey, z + ez
        ok = fluid.copy()
        for c, n, per in ((xn, nx, periodic[0]), (yn, ny, periodic[1]), (zn, nz, periodic[2])):
            if per:
                c %= n
            else:
                ok &= (c >= 0) & (c < n)
        nb = np.zeros_like(idx)
        nb[ok] = (xn[ok] + nx * (yn[ok] + ny * zn[ok])).astype(np.int64)
        hit = ok.copy()
        hit[ok] = solid[nb[ok]]
        nodes.append(idx[hit])
        dirs.append(np.full(np.count_nonzero(hit), i, np.uint8))
    nodes = np.concatenate(nodes)
    dirs = np.concatenate(dirs)
    order = np.lexsort((dirs, nodes))
    nodes, dirs = nodes[order], dirs[order]
    pts = np.stack([x[nodes], y[nodes], z[nodes]], axis=1)
    q = qfun(pts, D3Q19_DIRS[dirs].astype(np.float64))
    if np.any(~np.isfinite(q)) or np.any(q < 0) or np.any(q > 1):
        raise ValueError("wall fraction q outside [0, 1]")
    return nodes, dirs, q


def _bisect_q(sdf, pts, dirs, iters=60):
    """Crossing fraction of sdf = 0 on p + t*e, t in (0, 1], with
    sdf(p) < 0 <= sdf(p + e)."""
    lo = np.zeros(len(pts))
    hi = np.ones(len(pts))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        inside = sdf(pts + mid[:, None] * dirs) < 0
        lo = np.where(inside, mid, lo)
        hi = np.where(inside, hi, mid)
    return 0.5 * (lo + hi)


def periodic_box(nx, ny, nz, body_force=(0.0, 0.0, 0.0)):
    """All-fluid box, periodic on every axis (no walls, no open faces)."""
    n = nx * ny * nz
    return Domain(nx, ny, nz, (True, True, True), np.zeros(n, np.uint8),
                  np.zeros(0, np.int64), np.zeros(0, np.uint8), np.zeros(0),
                  np.zeros(0), 1.0, None, None, tuple(body_force),
                  meta={"kind": "periodic_box"})


def pipe(nx, ny, nz, radius, u_max=0.0, tau=0.8, periodic_x=False, init="poiseuille",
         body_force=(0.0, 0.0, 0.0), center=None):
    """Straight circular pipe along x.  Solid where r >= radius.

    Open ends (``periodic_x`` False): x = 0 is a velocity inlet carrying the
    parabolic profile u_max (1 - r^2/R^2) and x = nx-1 a density outlet at
    rho = 1.  ``init='poiseuille'`` starts from that profile with the linear
    Hagen-Poiseuille density drop towards the outlet (p = rho/3, nu from tau);
    ``init='rest'`` starts from rho = 1, u = 0.
    """
    yc, zc = center if center is not None else ((ny - 1) / 2.0, (nz - 1) / 2.0)
    x, y, z = _coords(nx, ny, nz)
    r2 = (y - yc) ** 2 + (z - zc) ** 2
    solid = r2 >= radius * radius
    periodic = (bool(periodic_x), False, False)
    nt = _tag_faces(nx, ny, nz, periodic, solid, inlet_faces=(0,))

    def qfun(pts, e):
        py, pz = pts[:, 1] - yc, pts[:, 2] - zc
        a = e[:, 1] ** 2 + e[:, 2] ** 2
        b = 2.0 * (py * e[:, 1] + pz * e[:, 2])
        c = py * py + pz * pz - radius * radius
        return (-b + np.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)

    ln, ld, lq = _links(nx, ny, nz, periodic, solid, qfun)
    prof = np.where(solid, 0.0, u_max * (1.0 - r2 / (radius * radius)))
    inlet = np.flatnonzero(nt == INLET)
    inlet_u = np.zeros((len(inlet), 3))
    inlet_u[:, 0] = prof[inlet]
    init_rho = init_u = None
    if init == "poiseuille":
        nu = (tau - 0.5) / 3.0
        init_u = np.zeros((3, nx * ny * nz))
        init_u[0] = prof
        if periodic_x:
            init_rho = np.ones(nx * ny * nz)
        else:
            init_rho = 1.0 + 12.0 * nu * u_max * ((nx - 1) - x) / (radius * radius)
        init_rho = np.where(solid, 1.0, init_rho)
        init_u = init_u.ravel()
    return Domain(nx, ny, nz, periodic, nt, ln, ld, lq, inlet_u.ravel(), 1.0,
                  init_rho, init_u, tuple(body_force),
                  meta={"kind": "pipe", "radius": radius, "center": (yc, zc),
                        "u_max": u_max, "tau": tau})


# ---------------------------------------------------------------- bifurcation
def _capped_cyl_sdf(a, b):
    """Signed distance of the intersection {a <= 0} & {b <= 0} of a radial and
    a cap coordinate (exact for a half-infinite cylinder)."""
    return np.minimum(np.maximum(a, b), 0.0) + np.hypot(np.maximum(a, 0.0), np.maximum(b, 0.0))


def _round_union(a, b, r):
    if r <= 0:
        return np.minimum(a, b)
    ua = np.maximum(r - a, 0.0)
    ub = np.maximum(r - b, 0.0)
    return np.maximum(r, np.minimum(a, b)) - np.hypot(ua, ub)


def bifurcation_sdf(params):
    """Signed distance (negative inside the fluid) of a symmetric
    Y-bifurcation in the x-y plane: a main tube along +x ending at the
    junction point J, and two daughter tubes leaving J along
    (cos t, +-sin t, 0), joined by rolling-ball fillets of radius ``fillet``.
    """
    R, Rd = params["R"], params["Rd"]
    J = np.asarray(params["J"], np.float64)
    th = params["theta"]
    fil = params["fillet"]
    d1 = np.array([np.cos(th), np.sin(th), 0.0])
    d2 = np.array([np.cos(th), -np.sin(th), 0.0])

    def sdf(p):
        p = np.atleast_2d(p)
        rel = p - J
        main = _capped_cyl_sdf(np.hypot(rel[:, 1], rel[:, 2]) - R, rel[:, 0])
        out = main
        dd = []
        for d in (d1, d2):
            t = rel @ d
            radial = np.linalg.norm(rel - t[:, None] * d[None, :], axis=1)
            dd.append(_capped_cyl_sdf(radial - Rd, -t))
        out = _round_union(_round_union(main, dd[0], fil), dd[1], fil)
        return out
    return sdf


def _edge_band_sdf(nx, ny, nz, band):
    """band - (distance to the nearest box edge), the distance to an edge
    being the larger of the distances to its two faces: positive (solid)
    within ``band`` of any of the twelve edges of the box."""
    def sdf(p):
        p = np.atleast_2d(p)
        dx = np.minimum(p[:, 0], nx - 1 - p[:, 0])
        dy = np.minimum(p[:, 1], ny - 1 - p[:, 1])
        dz = np.minimum(p[:, 2], nz - 1 - p[:, 2])
        d = np.minimum(np.minimum(np.maximum(dx, dy), np.maximum(dx, dz)), np.maximum(dy, dz))
        return band - d
    return sdf


def _junction_chamber_sdf(params):
    """The smooth junction: a prism whose section in the plane of the
    bifurcation is a trapezoid, from the end of the main tube (x = x_j) to a
    flat wall at x_j + H, H = Rd / sin(theta) + Rd (one daughter radius past
    the apex of the sharp junction, where the daughters' inner walls meet),
    its sides along the daughters' outer walls, its thickness the daughters'
    diameter.  The value is the largest signed distance to its bounding
    planes (exact in sign, a lower bound in size)."""
    Rd = params["Rd"]
    J = np.asarray(params["J"], np.float64)
    th = params["theta"]
    H = Rd / np.sin(th) + Rd
    sl = np.tan(th) if th < np.pi / 2 - 1e-9 else None
    cth = np.cos(th)

    def sdf(p):
        p = np.atleast_2d(p)
        rel = p - J
        xp, yp, zp = rel[:, 0], np.abs(rel[:, 1]), np.abs(rel[:, 2])
        d = np.maximum(-xp, xp - H)
        d = np.maximum(d, zp - Rd)
        if sl is not None:
            # side plane y = x tan(theta) + Rd / cos(theta), unit normal
            # (-sin(theta), cos(theta))
            d = np.maximum(d, (yp - xp * sl - Rd / cth) * cth)
        return d
    return sdf


def bifurcation(nx, ny, nz, D, daughter_ratio=0.8, theta_deg=60.0, fillet=4.0,
                x_junction=None, u_max=0.0, init="rest", edge_band=0.0, junction="sharp"):
    """Symmetric Y-bifurcation: main tube of diameter D along x centred at
    (y, z) = ((ny-1)/2, (nz-1)/2), junction at x = x_junction (default nx/2),
    daughters of diameter daughter_ratio*D at the semi-aperture angle
    theta (between the main axis and each daughter axis).

    x = 0 is a velocity inlet with the parabolic profile of peak u_max; every
    other fluid node on the box boundary is a density outlet (rho = 1).
    ``init='rest'`` starts from rho = 1, u = 0.  ``edge_band > 0`` makes the
    nodes within that distance of a box edge solid (a daughter tube leaving
    through a box edge would otherwise put open-boundary nodes on two faces);
    the wall there is a plane of the band, with its own link fractions.
    ``junction='smooth'`` replaces the sharp apex between the daughters by
    the flat wall of a trapezoidal chamber (the paper's two junctions).
    """
    yc, zc = (ny - 1) / 2.0, (nz - 1) / 2.0
    xj = nx / 2.0 if x_junction is None else x_junction
    params = {"R": D / 2.0, "Rd": daughter_ratio * D / 2.0, "J": (xj, yc, zc),
              "theta": np.deg2rad(theta_deg), "fillet": fillet, "junction": junction}
    sdf = bifurcation_sdf(params)
    if junction == "smooth":
        tubes, chamber = sdf, _junction_chamber_sdf(params)

        def sdf(p):
            return np.minimum(tubes(p), chamber(p))
    elif junction != "sharp":
        raise ValueError("junction: 'sharp' or 'smooth'")
    if edge_band > 0.0:
        tube, band = sdf, _edge_band_sdf(nx, ny, nz, edge_band)

        def sdf(p):
            return np.maximum(tube(p), band(p))
    x, y, z = _coords(nx, ny, nz)
    pts = np.stack([x, y, z], axis=1)
    solid = sdf(pts) >= 0.0
    periodic = (False, False, False)
    nt = _tag_faces(nx, ny, nz, periodic, solid, inlet_faces=(0,))
    ln, ld, lq = _links(nx, ny, nz, periodic, solid, lambda p, e: _bisect_q(sdf, p, e))
    R = D / 2.0
    r2 = (y - yc) ** 2 + (z - zc) ** 2
    inlet = np.flatnonzero(nt == INLET)
    inlet_u = np.zeros((len(inlet), 3))
    inlet_u[:, 0] = np.maximum(u_max * (1.0 - r2[inlet] / (R * R)), 0.0)
    init_rho = init_u = None
    if init != "rest":
        raise ValueError("bifurcation supports init='rest' only")
    return Domain(nx, ny, nz, periodic, nt, ln, ld, lq, inlet_u.ravel(), 1.0,
                  init_rho, init_u, (0.0, 0.0, 0.0),
                  meta={"kind": "bifurcation", "params": params, "u_max": u_max,
                        "sdf": sdf})
