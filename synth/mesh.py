"""Closed triangulated capsule meshes and their material parameters.

The icosphere starts from the regular icosahedron whose 12 vertices are the
cyclic permutations of (0, +-1, +-phi) (phi the golden ratio) and splits every
triangle into four by its edge midpoints, pushed back onto the sphere, ``subdiv``
times: 12 + 10*(4^s - 1) vertices and 20*4^s faces (s = 2: 162/320,
s = 3: 642/1280, s = 4: 2562/5120).  Faces are ordered counter-clockwise seen
from outside, so (b - a) x (c - a) points outward.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


# Fixed generic orientation (rotations of 1.1, 0.7 and 0.3 rad about x, y
# and z, in that order) applied by ``icosphere(..., tilt=True)``.  It keeps
# mesh vertices and face centroids of a sphere centred on a half-integer
# lattice coordinate off the planes where the nearest-node stencil base
# floor(x + 1/2) changes.
def _tilt_matrix():
    ax, ay, az = 1.1, 0.7, 0.3
    rx = np.array([[1, 0, 0], [0, np.cos(ax), -np.sin(ax)], [0, np.sin(ax), np.cos(ax)]])
    ry = np.array([[np.cos(ay), 0, np.sin(ay)], [0, 1, 0], [-np.sin(ay), 0, np.cos(ay)]])
    rz = np.array([[np.cos(az), -np.sin(az), 0], [np.sin(az), np.cos(az), 0], [0, 0, 1]])
    return rz @ ry @ rx


def icosphere(subdiv: int, radius: float = 1.0, center=(0.0, 0.0, 0.0), tilt: bool = False):
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0),
         (0, -1, phi), (0, 1, phi), (0, -1, -phi), (0, 1, -phi),
         (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    X = np.array(verts)
    F = np.array(faces, np.int32)
    # orient every face outward
    a, b, c = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    if tilt:
        X = X @ _tilt_matrix().T
    return X * radius + np.asarray(center, np.float64), F


def off_switch_planes(X, F, eps=1e-6):
    """True when no vertex and no face centroid lies within eps of a plane
    x_a = k + 1/2, where the 3x3x3 support base floor(x + 1/2) jumps: a marker
    released on such a plane has a support chosen by rounding."""
    for P in (X, X[F].mean(1)):
        fr = (P + 0.5) - np.floor(P + 0.5)
        if np.any((fr < eps) | (fr > 1.0 - eps)):
            return False
    return True


@dataclass
class Body:
    """A capsule: closed outward-oriented triangle mesh plus material
    parameters in the paper's terms.

    ``ca``     capillary number (stiffness from rho*nu*u_ref/Ca, rho = 1)
    ``eb``     bending number (k_b relative to the edge stiffness and r_ref^2)
    ``kv``     volume-penalty constant (<= 0: library default)
    ``rho_ratio`` solid/fluid density ratio, ``r_ref`` capsule radius,
    ``u_ref``  reference velocity in the capillary number,
    ``rigid``  rigid (Newton-Euler) instead of deformable,
    ``fixed``  held in place (prescribed zero velocity), rigid only.
    """
    x: np.ndarray          # float64 [nv, 3]
    faces: np.ndarray      # int32 [nf, 3]
    rigid: bool = False
    fixed: bool = False
    ca: float = 0.01
    eb: float = 0.001
    kv: float = -1.0
    rho_ratio: float = 1.1
    r_ref: float = 1.0
    u_ref: float = 0.0
    v0: np.ndarray | None = None

    @property
    def nv(self):
        return len(self.x)

    @property
    def nf(self):
        return len(self.faces)
