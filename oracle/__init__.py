"""ctypes binding of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB_PATH = os.path.join(_HERE, "liboracle.so")
LIB_PATH = DEFAULT_LIB_PATH
_lib = None


# Measurement builds of the same source, used only to gauge how far a
# trajectory moves under other rounding: "fma" lets the compiler fuse
# multiply-adds, "reassoc" lets it reorder sums (vectorised reductions),
# "store_f32" and "store_f16" round the stored populations to FP32 or to
# binary16; "ldouble" runs the fluid state and arithmetic in long double (a
# near-exact reference trajectory); "fullpop" stores full populations f
# instead of the deviations f - w ("fullpop_ldouble": both); "float" runs the
# fluid state and arithmetic in binary32; "fma_reassoc" both fma and reassoc.
VARIANT_FLAGS = {
    "plain": [],
    "fma": ["-mfma", "-ffp-contract=fast"],
    "reassoc": ["-O3", "-mavx2", "-fassociative-math", "-fno-signed-zeros", "-fno-trapping-math"],
    "store_f32": ["-DORC_STORE_F32"],
    "store_f16": ["-DORC_STORE_F16"],
    "ldouble": ["-DORC_LDOUBLE"],
    "fullpop": ["-DORC_FULL_POP"],
    "fullpop_ldouble": ["-DORC_FULL_POP", "-DORC_LDOUBLE"],
    "float": ["-DORC_FLOAT"],
    "fma_reassoc": ["-mfma", "-ffp-contract=fast", "-O3", "-mavx2", "-fassociative-math",
                    "-fno-signed-zeros", "-fno-trapping-math"],
}


def build(verbose=False, variant="plain", path=None):
    """Compile the oracle with the host compiler (gcc, OpenMP).  The default
    build is the oracle; a named variant goes to ``path``."""
    out = path or DEFAULT_LIB_PATH
    if variant != "plain" and path is None:
        raise ValueError("a measurement variant needs its own path")
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           *VARIANT_FLAGS[variant], os.path.join(_HERE, "oracle.c"), "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def use_library(path):
    """Load the oracle from ``path`` (a measurement build) in this process;
    must be called before the first use."""
    global LIB_PATH
    if _lib is not None:
        raise RuntimeError("oracle library already loaded")
    LIB_PATH = path


def _P(t):
    return C.POINTER(t)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if LIB_PATH != DEFAULT_LIB_PATH:
            raise FileNotFoundError(LIB_PATH)
        build()
    L = C.CDLL(LIB_PATH)
    d, i32, i64, u8 = C.c_double, C.c_int32, C.c_int64, C.c_uint8
    vp = C.c_void_p
    L.orc_create.restype = vp
    L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, _P(i32), d, d, _P(d), _P(u8), i64,
                             _P(i64), _P(u8), _P(d), _P(d), d, _P(d), _P(d), C.c_char_p, C.c_int]
    L.orc_destroy.argtypes = [vp]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_threads.restype = C.c_int
    L.orc_add_body.restype = C.c_int
    L.orc_add_body.argtypes = [vp, C.c_int, C.c_int, _P(d), _P(i32), C.c_int, C.c_int, d, d, d,
                               d, d, d, _P(d)]
    L.orc_step.restype = C.c_int
    L.orc_step.argtypes = [vp, C.c_int]
    L.orc_steps_done.restype = i64
    L.orc_steps_done.argtypes = [vp]
    L.orc_status.restype = C.c_int
    L.orc_status.argtypes = [vp]
    L.orc_mls_singular_count.restype = C.c_int
    L.orc_mls_singular_count.argtypes = [vp]
    for name in ("orc_get_fields",):
        getattr(L, name).argtypes = [vp, _P(d), _P(d)]
    L.orc_get_populations.argtypes = [vp, _P(d)]
    L.orc_get_populations_at.argtypes = [vp, i64, _P(i64), _P(d)]
    L.orc_set_populations.argtypes = [vp, _P(d)]
    L.orc_get_force.argtypes = [vp, _P(d)]
    L.orc_get_body.argtypes = [vp, C.c_int, _P(d), _P(d)]
    L.orc_body_diag.argtypes = [vp, C.c_int, _P(d)]
    L.orc_ib_interpolate.argtypes = [vp, i64, _P(d), _P(d), _P(d)]
    L.orc_ib_spread.argtypes = [vp, i64, _P(d), _P(d), _P(d), _P(d)]
    L.orc_mls_point.restype = C.c_int
    L.orc_mls_point.argtypes = [vp, _P(d), _P(i64), _P(d)]
    L.orc_lattice.argtypes = [_P(i32), _P(d)]
    L.orc_feq.argtypes = [d, _P(d), _P(d)]
    L.orc_guo.argtypes = [d, _P(d), _P(d), _P(d)]
    L.orc_bfl.restype = d
    L.orc_bfl.argtypes = [d, d, d, d, d, d, C.c_int, C.c_int]
    L.orc_zouhe.restype = d
    L.orc_zouhe.argtypes = [_P(d), C.c_int, C.c_int, _P(d), d]
    L.orc_membrane.restype = d
    L.orc_membrane.argtypes = [vp, C.c_int, _P(d), C.c_int, _P(d)]
    L.orc_body_hydro.argtypes = [vp, C.c_int, _P(d)]
    L.orc_body_fext.argtypes = [vp, C.c_int, _P(d)]
    L.orc_body_inertia.argtypes = [vp, C.c_int, _P(d)]
    L.orc_rodrigues.argtypes = [_P(d), _P(d)]
    L.orc_move_rigid.restype = C.c_int
    L.orc_move_rigid.argtypes = [vp, C.c_int, _P(d)]
    _lib = L
    return L


def _ptr(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(t))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------ element helpers
def lattice():
    e = np.zeros(57, np.int32)
    w = np.zeros(19)
    lib().orc_lattice(_ptr(e, C.c_int32), _ptr(w, C.c_double))
    return e.reshape(19, 3), w


def feq(rho, u):
    u = _f64(u)
    out = np.zeros(19)
    lib().orc_feq(rho, _ptr(u, C.c_double), _ptr(out, C.c_double))
    return out


def guo(tau, u, F):
    u, F = _f64(u), _f64(F)
    out = np.zeros(19)
    lib().orc_guo(tau, _ptr(u, C.c_double), _ptr(F, C.c_double), _ptr(out, C.c_double))
    return out


def bfl(q, fi_x, fi_xm1, fi_xm2, fj_x, fj_xm1, avail1=True, avail2=True):
    return lib().orc_bfl(q, fi_x, fi_xm1, fi_xm2, fj_x, fj_xm1, int(avail1), int(avail2))


def zouhe(f19, face, kind, u_w=(0.0, 0.0, 0.0), rho_w=1.0):
    f = np.array(f19, dtype=np.float64)
    uw = _f64(np.asarray(u_w, np.float64))
    r = lib().orc_zouhe(_ptr(f, C.c_double), face, kind, _ptr(uw, C.c_double), rho_w)
    return f, r


# ------------------------------------------------------------------ simulation
class OracleSim:
    """A full oracle simulation built from a ``synth`` domain (and bodies)."""

    def __init__(self, domain, tau, u_max=0.0, bodies=(), threads=None):
        L = lib()
        if threads is not None:
            L.orc_set_threads(int(threads))
        d = domain
        self.nx, self.ny, self.nz = d.nx, d.ny, d.nz
        self.N = d.nx * d.ny * d.nz
        per = np.array([int(p) for p in d.periodic], np.int32)
        g = _f64(np.asarray(d.body_force, np.float64))
        nt = np.ascontiguousarray(d.node_type, np.uint8)
        ln = np.ascontiguousarray(d.link_node, np.int64)
        ld = np.ascontiguousarray(d.link_dir, np.uint8)
        lq = _f64(d.link_q)
        iu = _f64(d.inlet_u) if len(d.inlet_u) else np.zeros(3)
        ir, iv = _f64(d.init_rho), _f64(d.init_u)
        err = C.create_string_buffer(256)
        self._h = L.orc_create(d.nx, d.ny, d.nz, _ptr(per, C.c_int32), tau, u_max, _ptr(g, C.c_double),
                               _ptr(nt, C.c_uint8), len(ln), _ptr(ln, C.c_int64), _ptr(ld, C.c_uint8),
                               _ptr(lq, C.c_double), _ptr(iu, C.c_double), d.outlet_rho,
                               _ptr(ir, C.c_double), _ptr(iv, C.c_double), err, 256)
        if not self._h:
            raise ValueError("oracle create failed: " + err.value.decode())
        self._destroy = lib().orc_destroy  # still reachable at interpreter exit
        self.tau = tau
        self.bodies = []
        for b in bodies:
            self.add_body(b)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def add_body(self, b):
        x = _f64(b.x)
        f = np.ascontiguousarray(b.faces, np.int32)
        v0 = _f64(b.v0)
        bid = lib().orc_add_body(self._h, len(x), len(f), _ptr(x, C.c_double), _ptr(f, C.c_int32),
                                 int(b.rigid), int(b.fixed), b.ca, b.eb, b.kv, b.rho_ratio,
                                 b.r_ref, b.u_ref, _ptr(v0, C.c_double))
        if bid < 0:
            raise ValueError(f"oracle add_body failed ({-bid})")
        self.bodies.append((len(x), len(f)))
        return bid

    def step(self, n=1):
        return lib().orc_step(self._h, int(n))

    @property
    def steps_done(self):
        return lib().orc_steps_done(self._h)

    @property
    def status(self):
        return lib().orc_status(self._h)

    @property
    def mls_singular(self):
        return lib().orc_mls_singular_count(self._h)

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        lib().orc_get_fields(self._h, _ptr(rho, C.c_double), _ptr(u, C.c_double))
        return rho, u.reshape(3, self.N)

    def populations(self):
        f = np.zeros(19 * self.N)
        lib().orc_get_populations(self._h, _ptr(f, C.c_double))
        return f.reshape(19, self.N)

    def set_populations(self, f):
        """The stored populations become f ([19][N]; solid entries ignored)."""
        f = _f64(np.asarray(f, np.float64).reshape(19 * self.N))
        lib().orc_set_populations(self._h, _ptr(f, C.c_double))

    def populations_at(self, nodes):
        """f_i at the listed node indices only, [19][len(nodes)]."""
        idx = np.ascontiguousarray(nodes, np.int64)
        f = np.zeros(19 * len(idx))
        lib().orc_get_populations_at(self._h, len(idx), _ptr(idx, C.c_int64), _ptr(f, C.c_double))
        return f.reshape(19, len(idx))

    def force(self):
        f = np.zeros(3 * self.N)
        lib().orc_get_force(self._h, _ptr(f, C.c_double))
        return f.reshape(3, self.N)

    def body(self, bid):
        nv, _ = self.bodies[bid]
        x = np.zeros(3 * nv)
        v = np.zeros(3 * nv)
        lib().orc_get_body(self._h, bid, _ptr(x, C.c_double), _ptr(v, C.c_double))
        return x.reshape(nv, 3), v.reshape(nv, 3)

    def body_diag(self, bid):
        o = np.zeros(20)
        lib().orc_body_diag(self._h, bid, _ptr(o, C.c_double))
        keys = ["V", "S", "V0", "S0", "max_strain", "mass", "kv", "ks0"]
        out = {k: o[i] for i, k in enumerate(keys)}
        out["xc"], out["u"], out["omega"] = o[8:11].copy(), o[11:14].copy(), o[14:17].copy()
        out["m_v"], out["rigid"], out["nf"] = o[17], o[18], o[19]
        return out

    def ib_interpolate(self, pts, field):
        pts = _f64(pts).reshape(-1, 3)
        field = _f64(field).reshape(3, self.N)
        out = np.zeros((len(pts), 3))
        lib().orc_ib_interpolate(self._h, len(pts), _ptr(pts, C.c_double), _ptr(field, C.c_double),
                                 _ptr(out, C.c_double))
        return out

    def ib_spread(self, pts, F, c):
        pts = _f64(pts).reshape(-1, 3)
        F = _f64(F).reshape(-1, 3)
        c = _f64(c).reshape(-1)
        out = np.zeros((3, self.N))
        lib().orc_ib_spread(self._h, len(pts), _ptr(pts, C.c_double), _ptr(F, C.c_double),
                            _ptr(c, C.c_double), _ptr(out, C.c_double))
        return out

    def mls_point(self, p):
        p = _f64(np.asarray(p, np.float64))
        node = np.zeros(27, np.int64)
        psi = np.zeros(27 * 4)
        ok = lib().orc_mls_point(self._h, _ptr(p, C.c_double), _ptr(node, C.c_int64), _ptr(psi, C.c_double))
        return bool(ok), node, psi.reshape(27, 4)

    def membrane(self, bid, x, which=7):
        x = _f64(x).reshape(-1, 3)
        F = np.zeros_like(x)
        E = lib().orc_membrane(self._h, bid, _ptr(x, C.c_double), int(which), _ptr(F, C.c_double))
        return E, F

    def body_hydro(self, bid):
        _, nf = self.bodies[bid]
        out = np.zeros((nf, 3))
        lib().orc_body_hydro(self._h, bid, _ptr(out, C.c_double))
        return out

    def body_fext(self, bid):
        """Per-face external force (hydrodynamic + repulsion) of the last step."""
        _, nf = self.bodies[bid]
        out = np.zeros((nf, 3))
        lib().orc_body_fext(self._h, bid, _ptr(out, C.c_double))
        return out

    def body_inertia(self, bid):
        """Body-frame inertia tensor of a body about its centre of mass."""
        out = np.zeros(9)
        lib().orc_body_inertia(self._h, bid, _ptr(out, C.c_double))
        return out.reshape(3, 3)

    def move_rigid(self, bid, Fv):
        """One rigid-body update of body bid with vertex forces Fv [nv, 3]."""
        return lib().orc_move_rigid(self._h, bid, _ptr(_f64(Fv), C.c_double))


def rodrigues(phi):
    """Rotation matrix of the rotation vector phi (the oracle's own)."""
    R = np.zeros(9)
    lib().orc_rodrigues(_ptr(_f64(phi), C.c_double), _ptr(R, C.c_double))
    return R.reshape(3, 3)


def from_workload(w, threads=None, with_bodies=True):
    return OracleSim(w.domain, w.tau, w.u_max, w.bodies if with_bodies else (), threads=threads)
