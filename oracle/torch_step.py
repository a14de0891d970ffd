"""The coupled step of the oracle written a second time, in PyTorch CPU FP64,
so that reverse-mode automatic differentiation of it gives the exact
discrete derivative of the step: the oracle's discrete adjoint.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (never by the product
package).  It shares no code with the GPU library and none with ``oracle.c``;
its forward trajectory is pinned against ``oracle.c``'s by the tests.

One step, in the paper's order (section "Numerical method and computational
procedure"), with the same readings as ``oracle.c``:
  S1 pull-streaming, interpolated bounce-back on wall links (Eq. bbouzidi,
     with the fallbacks where x - e_i or x - 2 e_i is unavailable);
  S2 Zou-He velocity / density faces (Eq. extbound, through direction
     vectors, the 1/6 terms carrying rho_w);
  S3 moments of the streamed populations, u* = sum f e / rho;
  S4 direct forcing at face centroids with moving-least-squares transfer
     (Eqs. uLag, l2norm, intKernel, the direct-forcing equation, bodyforce):
     3x3x3 support around floor(x + 1/2), W = exp(-(r/0.3)^2), r = |d| / 2.6,
     linear basis, c_l = face area;
  S5 BGK collision with the forcing term (Eqs. evoleq, eqfunc, forcing),
     populations as deviations f - w;
  S6 membrane forces as minus the gradient of the membrane energy (stretching
     1/2 k (l - l0)^2 per edge, bending k_b (1 - cos(theta - theta0)) per
     hinge, volume 1/2 (k_v / V0)(V - V0)^2), taken here by automatic
     differentiation of the energy;
  S7 hydrodynamic tractions from MLS fits at x_f +- 1.2 n (Eqs. hydroForP,
     hydroForNu);
  S8 Verlet with the MLS tentative velocity (Eqs. verletPos, verletVel,
     verletPosC).
Soft bodies only; no repulsion (one body, or bodies farther apart than dx).

Differentiable inputs: the initial post-collision deviations g0 [19, N], the
initial body state (positions P0, previous positions Q0, velocities V0, all
[nv, 3]), the inlet-velocity scale s (every inlet wall velocity times s), the
stiffness scale kappa (the membrane modulus k_s0 times kappa, with the
stretching, bending and default volume constants following it), the uniform
body force F [3] and the relaxation time tau (k_s0 held fixed).
"""
from __future__ import annotations

import numpy as np
import torch

# Eq. e_i and the weights that follow Eq. eqfunc
E = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [1, -1, 0], [1, 0, 1], [1, 0, -1], [-1, 1, 0], [-1, -1, 0], [-1, 0, 1],
              [-1, 0, -1], [0, 1, 1], [0, 1, -1], [0, -1, 1], [0, -1, -1]], np.int64)
WGT = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP = np.array([int(np.flatnonzero((E == -E[i]).all(1))[0]) for i in range(19)])
SOLID, INLET, OUTLET = 1, 2, 3
MLS_DEN = 2.6 * 2.6 * 0.09  # W = exp(-|d|^2 / (2.6^2 0.3^2))
DT = torch.float64


class TorchSim:
    """A coupled simulation from a ``synth`` workload, in torch FP64."""

    def __init__(self, w):
        d = w.domain
        self.nx, self.ny, self.nz = d.nx, d.ny, d.nz
        self.N = N = d.nx * d.ny * d.nz
        self.per = tuple(bool(p) for p in d.periodic)
        self.type = np.asarray(d.node_type, np.uint8)
        self.open = (self.type != SOLID)
        self.tau0 = float(w.tau)
        self.g0_force = np.asarray(d.body_force, np.float64)
        self._pull_plan(d)
        self._zouhe_plan(d)
        # initial populations: equilibrium of the initial fields
        rho0 = np.ones(N) if d.init_rho is None else np.asarray(d.init_rho, np.float64)
        u0 = np.zeros((3, N)) if d.init_u is None else np.asarray(d.init_u, np.float64).reshape(3, N)
        with torch.no_grad():
            g = self.feq_dev(torch.tensor(rho0, dtype=DT), torch.tensor(u0, dtype=DT))
            self.g_init = g * torch.tensor(self.open, dtype=DT)
        self.bodies = [self._body(b, w) for b in w.bodies]

    # ------------------------------------------------------------- geometry
    def _nbr(self, n, e):
        """Neighbour index of nodes n along integer offsets e [M, 3] (or one
        offset); -1 where it leaves the box through a non-periodic face."""
        nx, ny, nz = self.nx, self.ny, self.nz
        x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
        e = np.broadcast_to(np.asarray(e), (len(n), 3))
        c = [x + e[:, 0], y + e[:, 1], z + e[:, 2]]
        ok = np.ones(len(n), bool)
        for a, dim in enumerate((nx, ny, nz)):
            if self.per[a]:
                c[a] = c[a] % dim
            else:
                ok &= (c[a] >= 0) & (c[a] < dim)
        idx = c[0] + nx * (c[1] + ny * c[2])
        return np.where(ok, idx, -1)

    def _pull_plan(self, d):
        """h_j(x) = sum_t coef[j, t, x] * g[pop[j, t, x], src[j, t, x]] for the
        pulls: plain, interpolated bounce-back (Eq. bbouzidi with the
        fallbacks), or unknown (open face: filled by Zou-He)."""
        N = self.N
        q_of = {}
        for n, dr, q in zip(np.asarray(d.link_node), np.asarray(d.link_dir), np.asarray(d.link_q)):
            q_of[(int(n), int(dr))] = float(q)
        pop = np.zeros((19, 3, N), np.int64)
        src = np.zeros((19, 3, N), np.int64)
        coef = np.zeros((19, 3, N))
        nodes = np.arange(N)
        solid = self.type == SOLID
        for j in range(19):
            if j == 0:
                pop[0, 0], src[0, 0], coef[0, 0] = 0, nodes, 1.0
                continue
            s = self._nbr(nodes, -E[j])
            for n in range(N):
                if solid[n]:
                    continue
                if s[n] < 0:
                    continue  # unknown: Zou-He
                if not solid[s[n]]:
                    pop[j, 0, n], src[j, 0, n], coef[j, 0, n] = j, s[n], 1.0
                    continue
                i = OPP[j]
                q = q_of[(n, i)]
                a1 = self._nbr(np.array([n]), -E[i])[0]
                a2 = self._nbr(np.array([n]), -2 * E[i])[0]
                av1 = a1 >= 0 and not solid[a1]
                av2 = a2 >= 0 and not solid[a2]
                if q < 0.5:
                    if av1 and av2:
                        terms = [(i, n, q * (1 + 2 * q)), (i, a1, 1 - 4 * q * q), (i, a2, -q * (1 - 2 * q))]
                    elif av1:
                        terms = [(i, n, 2 * q), (i, a1, 1 - 2 * q)]
                    else:
                        terms = [(i, n, 1.0)]
                else:
                    if av1:
                        terms = [(i, n, 1 / (q * (2 * q + 1))), (j, n, (2 * q - 1) / q),
                                 (j, a1, (1 - 2 * q) / (1 + 2 * q))]
                    else:
                        terms = [(i, n, 1 / (2 * q)), (j, n, (2 * q - 1) / (2 * q))]
                for t, (pp, ss, cc) in enumerate(terms):
                    pop[j, t, n], src[j, t, n], coef[j, t, n] = pp, ss, cc
        self.flat = torch.tensor(pop * N + src, dtype=torch.int64)
        self.coef = torch.tensor(coef, dtype=DT)

    def _zouhe_plan(self, d):
        """Open nodes grouped by (face, kind) with their imposed values."""
        N = self.N
        nx, ny, nz = self.nx, self.ny, self.nz
        nodes = np.arange(N)
        x, y, z = nodes % nx, (nodes // nx) % ny, nodes // (nx * ny)
        uin = np.zeros((N, 3))
        inl = np.flatnonzero(self.type == INLET)
        if len(inl):
            uin[inl] = np.asarray(d.inlet_u, np.float64).reshape(-1, 3)
        self.groups = []
        for face in range(6):
            ax, hi = face // 2, face % 2
            if self.per[ax]:
                continue
            c = (x, y, z)[ax]
            on = c == ((nx, ny, nz)[ax] - 1 if hi else 0)
            nrm = np.zeros(3, np.int64)
            nrm[ax] = -1 if hi else 1
            for kind, tag in ((0, INLET), (1, OUTLET)):
                sel = np.flatnonzero(on & (self.type == tag))
                if len(sel):
                    self.groups.append((nrm, kind, torch.tensor(sel), torch.tensor(uin[sel].T, dtype=DT)))
        self.rho_out = float(d.outlet_rho)

    def _body(self, b, w):
        X = np.asarray(b.x, np.float64)
        F = np.asarray(b.faces, np.int64)
        nv = len(X)
        # edges (a -> b as in the first face that has it) and hinges
        first, second = {}, {}
        for f, (p, q, r) in enumerate(F):
            for a, c in ((p, q), (q, r), (r, p)):
                if (c, a) in first:
                    second[(c, a)] = f
                else:
                    first[(a, c)] = f
        edges, hinges = [], []
        for (a, c), f1 in first.items():
            f2 = second[(a, c)]
            wa = [v for v in F[f1] if v not in (a, c)][0]
            wd = [v for v in F[f2] if v not in (a, c)][0]
            edges.append((a, c, f1, f2))
            hinges.append((a, c, wa, wd))
        edges = np.array(edges, np.int64)
        hinges = np.array(hinges, np.int64)
        Xt = torch.tensor(X, dtype=DT)
        cen, nrm, area = face_geom(Xt, torch.tensor(F))
        nu0 = (self.tau0 - 0.5) / 3.0
        ks0 = nu0 * b.u_ref / b.ca
        l0 = (Xt[edges[:, 0]] - Xt[edges[:, 1]]).norm(dim=1)
        kl = ks0 * (area[edges[:, 2]] + area[edges[:, 3]]) / (l0 * l0)
        kb = b.eb * kl * b.r_ref ** 2
        with torch.no_grad():
            th0 = dihedral(Xt, torch.tensor(hinges))
        V0 = float(mesh_volume(Xt, torch.tensor(F)))
        kv_fixed = b.kv if b.kv > 0 else None
        v0 = np.zeros_like(X) if b.v0 is None else np.asarray(b.v0, np.float64)
        return dict(F=torch.tensor(F), edges=torch.tensor(edges[:, :2]), hinges=torch.tensor(hinges),
                    l0=l0.detach(), kl=kl.detach(), kb=kb.detach(), th0=th0, V0=V0, ks0=ks0,
                    kv_fixed=kv_fixed, r=b.r_ref, m_v=b.rho_ratio * V0 / nv,
                    P0=Xt.clone(), Q0=torch.tensor(X - v0, dtype=DT), V0v=torch.tensor(v0, dtype=DT))

    # ----------------------------------------------------------- fluid parts
    def feq_dev(self, rho, u):
        """Eq. eqfunc as deviations f^eq - w: [19, N]."""
        e = torch.tensor(E.T, dtype=DT)  # [3, 19]
        eu = (e.T @ u)                    # [19, N]
        uu = (u * u).sum(0)
        w = torch.tensor(WGT, dtype=DT)[:, None]
        return w * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu))

    def stream(self, g, s):
        """S1 + S2: streamed deviations h [19, N]."""
        h = (self.coef * g.reshape(-1)[self.flat]).sum(1)
        h = h * torch.tensor(self.open, dtype=DT)
        for nrm, kind, sel, uin in self.groups:
            h = self._zouhe(h, nrm, kind, sel, uin, s)
        return h

    def _zouhe(self, h, n, kind, sel, uin, s):
        en = E @ n
        d = h[:, sel]
        D0 = d[en == 0].sum(0)
        Dout = d[en == -1].sum(0)
        nt = torch.tensor(n, dtype=DT)
        if kind == 0:
            uw = s * uin
            un = (uw * nt[:, None]).sum(0)
            rho_w = (1.0 + D0 + 2.0 * Dout) / (1.0 - un)
        else:
            rho_w = torch.full_like(D0, self.rho_out)
            un = (rho_w - 1.0 - D0 - 2.0 * Dout) / rho_w
            uw = un[None, :] * nt[:, None]
        rows = list(d)
        for j in np.flatnonzero(en == 1):
            jb = OPP[j]
            t = E[j] - n
            if not t.any():
                rows[j] = d[jb] + rho_w / 3.0 * un
            else:
                ut = (uw * torch.tensor(t, dtype=DT)[:, None]).sum(0)
                Nt = sum(d[k] * float(E[k] @ t) for k in np.flatnonzero(en == 0))
                Nt = 0.5 * Nt - rho_w / 3.0 * ut
                rows[j] = d[jb] + rho_w / 6.0 * (un + ut) - Nt
        h = h.clone()
        h[:, sel] = torch.stack(rows)
        return h

    def collide(self, h, rho, m, Ftot, tau):
        """S5 on all nodes (solid rows are zeroed by the caller)."""
        u = (m + 0.5 * Ftot) / rho
        e = torch.tensor(E.T, dtype=DT)
        eu = e.T @ u
        w = torch.tensor(WGT, dtype=DT)[:, None]
        guo = (1.0 - 1.0 / (2.0 * tau)) * w * (3.0 * (e.T @ Ftot - (u * Ftot).sum(0)) + 9.0 * eu * (e.T @ Ftot))
        g = h - (h - self.feq_dev(rho, u)) / tau + guo
        return g, u

    # ------------------------------------------------------------------ MLS
    def mls(self, p):
        """Supports and coefficient weights of points p [M, 3]: node index
        [M, 27] (valid ones), mask [M, 27], psi [M, 27, 4] with psi[..., 0] the
        interpolation weight phi and psi[..., 1:] the gradient of the fit."""
        base = torch.floor(p.detach() + 0.5).to(torch.int64)
        k = np.arange(27)
        off = torch.tensor(np.stack([k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1], 1))
        c = base[:, None, :] + off[None]
        dims = (self.nx, self.ny, self.nz)
        ok = torch.ones(c.shape[:2], dtype=torch.bool)
        cw = c.clone()
        for a in range(3):
            if self.per[a]:
                cw[..., a] = cw[..., a] % dims[a]
            else:
                ok &= (c[..., a] >= 0) & (c[..., a] < dims[a])
        idx = cw[..., 0] + self.nx * (cw[..., 1] + self.ny * cw[..., 2])
        idx = torch.where(ok, idx, torch.zeros_like(idx))
        ok &= torch.tensor(self.type != SOLID)[idx]
        dv = c.to(DT) - p[:, None, :]
        W = torch.exp(-(dv * dv).sum(-1) / MLS_DEN) * ok.to(DT)
        P = torch.cat([torch.ones_like(dv[..., :1]), dv], -1)           # [M, 27, 4]
        A = torch.einsum("mk,mki,mkj->mij", W, P, P)
        Ainv = torch.linalg.inv(A)
        psi = W[..., None] * torch.einsum("mij,mkj->mki", Ainv, P)
        return idx, ok, psi

    # ---------------------------------------------------------------- step
    def step(self, st, prm):
        """One coupled step.  st = dict(g, bodies=[(P, Q, V)]); prm = dict(s,
        kappa, F, tau).  Returns the new state and the step's rho, u."""
        g, tau = st["g"], prm["tau"]
        N = self.N
        openm = torch.tensor(self.open, dtype=DT)
        h = self.stream(g, prm["s"])
        e = torch.tensor(E, dtype=DT)
        rho = 1.0 + h.sum(0)
        m = e.T @ h
        ustar = m / rho
        fib = torch.zeros(3, N, dtype=DT)
        for B, (P, Q, V) in zip(self.bodies, st["bodies"]):
            cen, nrm, area = face_geom(P, B["F"])
            idx, ok, psi = self.mls(cen)
            phi = psi[..., 0] * ok.to(DT)
            U = torch.einsum("mk,amk->ma", phi, ustar[:, idx])
            Ub = V[B["F"]].mean(1)
            Fl = Ub - U
            contrib = (area[:, None, None] * phi[..., None] * Fl[:, None, :]).reshape(-1, 3)
            fib = fib.index_add(1, idx.reshape(-1), contrib.T)
        Ftot = prm["F"][:, None] + fib
        gn, u = self.collide(h, rho, m, Ftot, tau)
        gn = gn * openm
        rho_o, u_o = rho * openm, u * openm
        nu = (tau - 0.5) / 3.0
        out_b = []
        for B, (P, Q, V) in zip(self.bodies, st["bodies"]):
            Fv = self.membrane_force(B, P, prm["kappa"]) + self.hydro_vertex(B, P, rho_o, u_o, nu)
            idx, ok, psi = self.mls(P)
            u0 = torch.einsum("mk,amk->ma", psi[..., 0] * ok.to(DT), u_o[:, idx])
            acc = 0.5 * Fv / B["m_v"]
            xt = P + u0 + acc
            Vn = 1.5 * xt - 2.0 * P + 0.5 * Q
            Pn = P + Vn + acc
            out_b.append((Pn, P, Vn))
        return {"g": gn, "bodies": out_b}, rho_o, u_o

    def membrane_force(self, B, P, kappa):
        """-grad of the membrane energy at P (kept differentiable)."""
        with torch.enable_grad():
            x = P if P.requires_grad else P.detach().requires_grad_(True)
            Es = 0.5 * (kappa * B["kl"] * ((x[B["edges"][:, 0]] - x[B["edges"][:, 1]]).norm(dim=1) - B["l0"]) ** 2).sum()
            th = dihedral(x, B["hinges"])
            Eb = (kappa * B["kb"] * (1.0 - torch.cos(th - B["th0"]))).sum()
            kv = B["kv_fixed"] if B["kv_fixed"] is not None else kappa * 10.0 * B["ks0"] / B["r"]
            V = mesh_volume(x, B["F"])
            Ev = 0.5 * kv / B["V0"] * (V - B["V0"]) ** 2
            (gx,) = torch.autograd.grad(Es + Eb + Ev, x, create_graph=True)
        return -gx

    def hydro_vertex(self, B, P, rho, u, nu):
        """S7: a third of each face's traction force at its vertices."""
        cen, nrm, area = face_geom(P, B["F"])
        fits = []
        for sg in (1.2, -1.2):
            idx, ok, psi = self.mls(cen + sg * nrm)
            okd = ok.to(DT)
            r = torch.einsum("mk,mk->m", psi[..., 0] * okd, rho[idx])
            G = torch.einsum("mkc,amk->mac", psi[..., 1:] * okd[..., None], u[:, idx])
            fits.append((r, G))
        (rp, Gp), (rm, Gm) = fits
        dp = (rp - rm) / 3.0
        tp = rp[:, None, None] * nu * (Gp + Gp.transpose(1, 2))
        tm = rm[:, None, None] * nu * (Gm + Gm.transpose(1, 2))
        tn = torch.einsum("mac,mc->ma", tp - tm, nrm)
        Ff = (-dp[:, None] * nrm + tn) * area[:, None]
        Fv = torch.zeros_like(P)
        for r in range(3):
            Fv = Fv.index_add(0, B["F"][:, r], Ff / 3.0)
        return Fv

    # ------------------------------------------------------------ running
    def initial_state(self):
        return {"g": self.g_init.clone(),
                "bodies": [(B["P0"].clone(), B["Q0"].clone(), B["V0v"].clone()) for B in self.bodies]}

    def params(self, s=1.0, kappa=1.0, F=None, tau=None):
        return {"s": torch.tensor(s, dtype=DT), "kappa": torch.tensor(kappa, dtype=DT),
                "F": torch.tensor(self.g0_force if F is None else F, dtype=DT),
                "tau": torch.tensor(self.tau0 if tau is None else tau, dtype=DT)}


def face_geom(X, F):
    a, b, c = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    N = torch.linalg.cross(b - a, c - a)
    l = N.norm(dim=1)
    return (a + b + c) / 3.0, N / l[:, None], 0.5 * l


def mesh_volume(X, F):
    a, b, c = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    return (a * torch.linalg.cross(b, c)).sum() / 6.0


def dihedral(X, H):
    """Signed angle between the outward normals of faces (a, b, c) and
    (b, a, d) of each hinge (a, b, c, d)."""
    a, b, c, d = X[H[:, 0]], X[H[:, 1]], X[H[:, 2]], X[H[:, 3]]
    e = b - a
    n1 = torch.linalg.cross(e, c - a)
    n2 = torch.linalg.cross(a - b, d - b)
    m1 = n1 / n1.norm(dim=1, keepdim=True)
    m2 = n2 / n2.norm(dim=1, keepdim=True)
    t = torch.linalg.cross(m1, m2)
    return torch.atan2((t * e).sum(1) / e.norm(dim=1), (m1 * m2).sum(1))


def taylor_deformation(P):
    """D_T = (sqrt(l1) - sqrt(l3)) / (sqrt(l1) + sqrt(l3)) from the largest
    and smallest eigenvalues of the vertex second-moment tensor."""
    d = P - P.mean(0)
    M = d.T @ d / P.shape[0]
    lam = torch.linalg.eigvalsh(M)
    a, c = torch.sqrt(lam[2]), torch.sqrt(lam[0])
    return (a - c) / (a + c)
