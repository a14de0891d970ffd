"""ctypes binding of the C ABI in ``include/lbm.h`` (argument marshalling
only: every step of the method runs in the gfx950 library).

Device buffers are torch tensors on the current HIP device; work is enqueued
on torch's current stream at context creation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmib.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_HIP, LBM_E_UNSTABLE, LBM_E_DAMAGED, LBM_E_STATE, \
    LBM_E_UNSUPPORTED = range(8)
STATUS_NAMES = {0: "OK", 1: "INVAL", 2: "NOMEM", 3: "HIP", 4: "UNSTABLE", 5: "DAMAGED",
                6: "STATE", 7: "UNSUPPORTED"}
PRECISIONS = {"f64": 0, "f32": 1, "f16s": 2}

# Every symbol the header declares (checked by the CPU test-suite).
EXPORTS = ["lbm_create", "lbm_destroy", "lbm_last_error", "lbm_info", "lbm_add_body", "lbm_step",
           "lbm_sync", "lbm_get_fields", "lbm_get_populations", "lbm_set_populations", "lbm_get_force",
           "lbm_get_body",
           "ib_interpolate", "ib_spread", "ib_spread_noalloc", "lbm_adjoint_step", "lbm_adjoint_run",
           "lbm_set_scales", "lbm_save", "lbm_load",
           "lbm_time_fluid_kernel", "lbm_set_graph", "lbm_set_launch_shape", "lbm_diagnostics",
           "lbm_batch_create",
           "lbm_batch_destroy", "lbm_batch_last_error", "lbm_batch_step", "lbm_batch_tune",
           "lbm_batch_set_shape", "lbm_batch_get_shape", "lbm_batch_time_fluid",
           "lbm_batch_set_graph"]


class LbmError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"lbm status {STATUS_NAMES.get(status, status)}: {msg}")


class LbmDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("tau", C.c_double), ("u_max", C.c_double),
                ("body_force", C.c_double * 3), ("precision", C.c_int32),
                ("node_type", C.POINTER(C.c_uint8)), ("n_links", C.c_int64),
                ("link_node", C.POINTER(C.c_int64)), ("link_dir", C.POINTER(C.c_uint8)),
                ("link_q", C.POINTER(C.c_double)), ("inlet_u", C.POINTER(C.c_double)),
                ("outlet_rho", C.c_double), ("init_rho", C.POINTER(C.c_double)),
                ("init_u", C.POINTER(C.c_double))]


class LbmBodyDesc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nf", C.c_int32), ("x", C.POINTER(C.c_double)),
                ("faces", C.POINTER(C.c_int32)), ("rigid", C.c_int32), ("fixed", C.c_int32),
                ("ca", C.c_double), ("eb", C.c_double), ("kv", C.c_double),
                ("rho_ratio", C.c_double), ("r_ref", C.c_double), ("u_ref", C.c_double),
                ("v0", C.POINTER(C.c_double))]


class LbmInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_fluid", C.c_int64), ("n_bulk", C.c_int64),
                ("n_general", C.c_int64), ("n_links", C.c_int64), ("n_bodies", C.c_int64),
                ("n_vertices", C.c_int64), ("n_faces", C.c_int64), ("steps_done", C.c_int64),
                ("bytes_per_step_alg", C.c_int64), ("precision", C.c_int32),
                ("mls_singular", C.c_int32), ("fluid_launch", C.c_int32), ("pad", C.c_int32)]


class LbmBatchShape(C.Structure):
    _fields_ = [("bulk_v", C.c_int32), ("block", C.c_int32), ("mode", C.c_int32),
                ("per_xcd", C.c_int32), ("fluid_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library():
    """Load liblbmib.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2207_06043_amd.build.build()")
    import torch  # noqa: F401  (load torch's HIP runtime first so both share it)
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    st = C.c_int
    L.lbm_create.restype = st
    L.lbm_create.argtypes = [C.POINTER(LbmDesc), vp, C.POINTER(vp)]
    L.lbm_destroy.restype = st
    L.lbm_destroy.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_last_error.argtypes = [vp]
    L.lbm_info.restype = st
    L.lbm_info.argtypes = [vp, C.POINTER(LbmInfo)]
    L.lbm_add_body.restype = st
    L.lbm_add_body.argtypes = [vp, C.POINTER(LbmBodyDesc), C.POINTER(i32)]
    L.lbm_step.restype = st
    L.lbm_step.argtypes = [vp, i32]
    L.lbm_sync.restype = st
    L.lbm_sync.argtypes = [vp]
    for name in ("lbm_get_fields",):
        getattr(L, name).restype = st
        getattr(L, name).argtypes = [vp, vp, vp]
    L.lbm_get_populations.restype = st
    L.lbm_get_populations.argtypes = [vp, vp]
    L.lbm_set_populations.restype = st
    L.lbm_set_populations.argtypes = [vp, vp]
    L.lbm_get_force.restype = st
    L.lbm_get_force.argtypes = [vp, vp]
    L.lbm_get_body.restype = st
    L.lbm_get_body.argtypes = [vp, i32, vp, vp]
    L.ib_interpolate.restype = st
    L.ib_interpolate.argtypes = [vp, i64, vp, vp, vp]
    L.ib_spread.restype = st
    L.ib_spread.argtypes = [vp, i64, vp, vp, vp, vp]
    L.ib_spread_noalloc.restype = st
    L.ib_spread_noalloc.argtypes = [vp, i64, vp, vp, vp, vp]
    L.lbm_adjoint_step.restype = st
    L.lbm_adjoint_step.argtypes = [vp, i32, i32, vp, vp, vp]
    L.lbm_adjoint_run.restype = st
    L.lbm_adjoint_run.argtypes = [vp, i32, i32, vp, C.c_double, i32, vp, vp, vp, dp]
    L.lbm_set_scales.restype = st
    L.lbm_set_scales.argtypes = [vp, C.c_double, C.c_double]
    L.lbm_save.restype = st
    L.lbm_save.argtypes = [vp, C.c_char_p]
    L.lbm_load.restype = st
    L.lbm_load.argtypes = [vp, C.c_char_p]
    L.lbm_time_fluid_kernel.restype = st
    L.lbm_time_fluid_kernel.argtypes = [vp, i32, dp]
    L.lbm_set_graph.restype = st
    L.lbm_set_graph.argtypes = [vp, i32]
    L.lbm_diagnostics.restype = st
    L.lbm_diagnostics.argtypes = [vp, dp]
    L.lbm_set_launch_shape.restype = st
    L.lbm_set_launch_shape.argtypes = [vp, i32, i32]
    L.lbm_batch_create.restype = st
    L.lbm_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
    L.lbm_batch_destroy.restype = st
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_last_error.restype = C.c_char_p
    L.lbm_batch_last_error.argtypes = [vp]
    L.lbm_batch_step.restype = st
    L.lbm_batch_step.argtypes = [vp, i32]
    L.lbm_batch_tune.restype = st
    L.lbm_batch_tune.argtypes = [vp, i32, C.POINTER(LbmBatchShape), i32, C.POINTER(i32)]
    L.lbm_batch_set_shape.restype = st
    L.lbm_batch_set_shape.argtypes = [vp, C.POINTER(LbmBatchShape)]
    L.lbm_batch_get_shape.restype = st
    L.lbm_batch_get_shape.argtypes = [vp, C.POINTER(LbmBatchShape)]
    L.lbm_batch_time_fluid.restype = st
    L.lbm_batch_time_fluid.argtypes = [vp, i32, dp]
    L.lbm_batch_set_graph.restype = st
    L.lbm_batch_set_graph.argtypes = [vp, i32]
    _lib = L
    return L


def _p(a, t):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


class Lattice:
    """One lattice context on the current HIP device (see ``include/lbm.h``)."""

    def __init__(self, domain, tau, u_max=0.0, precision="f64", stream=None):
        import torch
        L = load_library()
        self._torch = torch
        d = domain
        self.nx, self.ny, self.nz = d.nx, d.ny, d.nz
        self.N = d.nx * d.ny * d.nz
        self.device = torch.device("cuda", torch.cuda.current_device())
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        keep = {}
        keep["nt"] = np.ascontiguousarray(d.node_type, np.uint8)
        keep["ln"] = np.ascontiguousarray(d.link_node, np.int64)
        keep["ld"] = np.ascontiguousarray(d.link_dir, np.uint8)
        keep["lq"] = np.ascontiguousarray(d.link_q, np.float64)
        keep["iu"] = np.ascontiguousarray(d.inlet_u if len(d.inlet_u) else np.zeros(3), np.float64)
        keep["ir"] = None if d.init_rho is None else np.ascontiguousarray(d.init_rho, np.float64)
        keep["iv"] = None if d.init_u is None else np.ascontiguousarray(d.init_u, np.float64)
        desc = LbmDesc()
        desc.nx, desc.ny, desc.nz = d.nx, d.ny, d.nz
        for a in range(3):
            desc.periodic[a] = int(bool(d.periodic[a]))
            desc.body_force[a] = float(d.body_force[a])
        desc.tau = float(tau)
        desc.u_max = float(u_max)
        desc.precision = PRECISIONS[precision]
        desc.node_type = _p(keep["nt"], C.c_uint8)
        desc.n_links = len(keep["ln"])
        desc.link_node = _p(keep["ln"], C.c_int64)
        desc.link_dir = _p(keep["ld"], C.c_uint8)
        desc.link_q = _p(keep["lq"], C.c_double)
        desc.inlet_u = _p(keep["iu"], C.c_double)
        desc.outlet_rho = float(d.outlet_rho)
        desc.init_rho = _p(keep["ir"], C.c_double)
        desc.init_u = _p(keep["iv"], C.c_double)
        h = C.c_void_p()
        s = L.lbm_create(C.byref(desc), C.c_void_p(stream.cuda_stream), C.byref(h))
        self._h = h
        if s != LBM_OK:
            msg = L.lbm_last_error(h).decode() if h.value else ""
            if h.value:
                L.lbm_destroy(h)
            self._h = None
            raise LbmError(s, msg)
        self.precision = precision
        self.bodies = []

    def _check(self, s):
        if s != LBM_OK:
            raise LbmError(s, load_library().lbm_last_error(self._h).decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                load_library().lbm_destroy(h)
            except Exception:
                pass
            self._h = None

    def close(self):
        self.__del__()

    # ---------------------------------------------------------------- bodies
    def add_body(self, b):
        L = load_library()
        x = np.ascontiguousarray(b.x, np.float64)
        f = np.ascontiguousarray(b.faces, np.int32)
        v0 = None if b.v0 is None else np.ascontiguousarray(b.v0, np.float64)
        bd = LbmBodyDesc()
        bd.nv, bd.nf = len(x), len(f)
        bd.x, bd.faces = _p(x, C.c_double), _p(f, C.c_int32)
        bd.rigid, bd.fixed = int(b.rigid), int(b.fixed)
        bd.ca, bd.eb, bd.kv = float(b.ca), float(b.eb), float(b.kv)
        bd.rho_ratio, bd.r_ref, bd.u_ref = float(b.rho_ratio), float(b.r_ref), float(b.u_ref)
        bd.v0 = _p(v0, C.c_double)
        bid = C.c_int32()
        self._check(L.lbm_add_body(self._h, C.byref(bd), C.byref(bid)))
        self.bodies.append((len(x), len(f)))
        return bid.value

    # ----------------------------------------------------------------- steps
    def step(self, n=1):
        self._check(load_library().lbm_step(self._h, int(n)))

    def sync(self, raise_on_stop=True):
        s = load_library().lbm_sync(self._h)
        if s in (LBM_E_UNSTABLE, LBM_E_DAMAGED) and not raise_on_stop:
            return s
        self._check(s)
        return s

    def set_graph(self, enable):
        self._check(load_library().lbm_set_graph(self._h, int(bool(enable))))

    def info(self):
        o = LbmInfo()
        self._check(load_library().lbm_info(self._h, C.byref(o)))
        return {k: getattr(o, k) for k, _ in LbmInfo._fields_}

    def diagnostics(self):
        """FP64 total mass and momentum of the last completed step, and per body
        (volume, surface, largest stretch) at the current positions."""
        out = (C.c_double * (4 + 3 * len(self.bodies)))()
        self._check(load_library().lbm_diagnostics(self._h, out))
        vals = list(out)
        return {"mass": vals[0], "momentum": vals[1:4],
                "bodies": [tuple(vals[4 + 3 * b: 7 + 3 * b]) for b in range(len(self.bodies))]}

    def set_launch_shape(self, bulk_v, block):
        self._check(load_library().lbm_set_launch_shape(self._h, int(bulk_v), int(block)))

    def time_fluid_kernel(self, n):
        ms = C.c_double()
        self._check(load_library().lbm_time_fluid_kernel(self._h, int(n), C.byref(ms)))
        return ms.value

    # --------------------------------------------------------------- outputs
    def _empty(self, *shape):
        return self._torch.empty(*shape, dtype=self._torch.float64, device=self.device)

    def fields(self):
        rho, u = self._empty(self.N), self._empty(3, self.N)
        self._check(load_library().lbm_get_fields(self._h, _ptr(rho), _ptr(u)))
        self.stream.synchronize()
        return rho, u

    def populations(self):
        f = self._empty(19, self.N)
        self._check(load_library().lbm_get_populations(self._h, _ptr(f)))
        self.stream.synchronize()
        return f

    def set_populations(self, f):
        """The current state's populations become f ([19][N]; see
        lbm_set_populations)."""
        f = f.to(self.device, self._torch.float64).reshape(19, self.N).contiguous()
        self._check(load_library().lbm_set_populations(self._h, _ptr(f)))
        self.stream.synchronize()

    def force(self):
        f = self._empty(3, self.N)
        self._check(load_library().lbm_get_force(self._h, _ptr(f)))
        self.stream.synchronize()
        return f

    def body(self, bid):
        nv, _ = self.bodies[bid]
        x, v = self._empty(nv, 3), self._empty(nv, 3)
        self._check(load_library().lbm_get_body(self._h, int(bid), _ptr(x), _ptr(v)))
        self.stream.synchronize()
        return x, v

    def ib_interpolate(self, pts, field=None):
        pts = pts.to(self.device, self._torch.float64).contiguous()
        out = self._empty(pts.shape[0], 3)
        fld = None if field is None else field.to(self.device, self._torch.float64).contiguous()
        self._check(load_library().ib_interpolate(self._h, pts.shape[0], _ptr(pts), _ptr(fld), _ptr(out)))
        self.stream.synchronize()
        return out

    def ib_spread(self, pts, F, c, fib=None):
        t = self._torch
        pts = pts.to(self.device, t.float64).contiguous()
        F = F.to(self.device, t.float64).contiguous()
        c = c.to(self.device, t.float64).contiguous()
        if fib is None:
            fib = t.zeros(3, self.N, dtype=t.float64, device=self.device)
        self._check(load_library().ib_spread(self._h, pts.shape[0], _ptr(pts), _ptr(F), _ptr(c), _ptr(fib)))
        self.stream.synchronize()
        return fib

    def ib_spread_noalloc(self, pts, F, c, fib):
        """The allocation-free spread: fib ([3][N] FP64 on the device) += the
        spread of c*F at pts; the caller supplies every buffer."""
        self._check(load_library().ib_spread_noalloc(self._h, pts.shape[0], _ptr(pts), _ptr(F), _ptr(c),
                                                     _ptr(fib)))
        return fib

    def adjoint(self, n_steps, lam, w=None, checkpoint_every=100):
        """Gradient of J = <lam, g^n> + sum_{t=1..n} <w, g^t> over the
        n_steps-step trajectory from the current state (g: the populations'
        deviations f - w_i, [19][N]); returns (dJ/dg^0 [19][N],
        [dJ/ds, dJ/dFx, dJ/dFy, dJ/dFz, dJ/dtau]) with s the inlet-velocity
        scale, F the body force and tau the relaxation time.  The lattice's
        state is not changed."""
        t = self._torch
        lam = lam.to(self.device, t.float64).reshape(19, self.N).clone()
        wd = None if w is None else w.to(self.device, t.float64).reshape(19, self.N).contiguous()
        grad = self._empty(5)
        self._check(load_library().lbm_adjoint_step(self._h, int(n_steps), int(checkpoint_every),
                                                    _ptr(wd), _ptr(lam), _ptr(grad)))
        self.stream.synchronize()
        return lam, grad

    def adjoint_run(self, n_steps, lam=None, w=None, taylor_weight=0.0, taylor_body=0,
                    checkpoint_every=100, body_grad=False):
        """lbm_adjoint_run: the gradient of J = <lam, g^n> + sum_t <w, g^t> +
        taylor_weight * sum_t D_T(body) over the n_steps-step trajectory from
        the current state.  Returns (dJ/dg^0 [19][N], [dJ/ds, dJ/dF (3),
        dJ/dtau, dJ/dkappa], dJ/d(x^0, x^{-1}, u_v^0) [3][nv][3] or None,
        (J's population part, the sum of D_T)).  The state is not changed."""
        t = self._torch
        if lam is None:
            lam = t.zeros(19, self.N, dtype=t.float64, device=self.device)
        lam = lam.to(self.device, t.float64).reshape(19, self.N).clone()
        wd = None if w is None else w.to(self.device, t.float64).reshape(19, self.N).contiguous()
        grad = self._empty(6)
        nv = sum(b[0] for b in self.bodies)
        bg = self._empty(3, nv, 3) if body_grad else None
        J = (C.c_double * 2)()
        self._check(load_library().lbm_adjoint_run(self._h, int(n_steps), int(checkpoint_every), _ptr(wd),
                                                   float(taylor_weight), int(taylor_body), _ptr(lam),
                                                   _ptr(grad), _ptr(bg), J))
        self.stream.synchronize()
        return lam, grad, bg, (J[0], J[1])

    def set_scales(self, inlet=1.0, stiffness=1.0):
        """lbm_set_scales: inlet wall velocities times `inlet`, membrane
        moduli times `stiffness` (relative to the lattice as created)."""
        self._check(load_library().lbm_set_scales(self._h, float(inlet), float(stiffness)))

    def save(self, path):
        self._check(load_library().lbm_save(self._h, str(path).encode()))

    def load(self, path):
        self._check(load_library().lbm_load(self._h, str(path).encode()))


class Batch:
    """Independent lattices advanced together (see ``include/lbm.h``, batching
    form).  The lattices must share precision and stream and outlive the
    batch; they keep working on their own."""

    def __init__(self, lattices):
        L = load_library()
        self.lattices = list(lattices)
        arr = (C.c_void_p * len(self.lattices))(*[lat._h.value for lat in self.lattices])
        h = C.c_void_p()
        s = L.lbm_batch_create(arr, len(self.lattices), C.byref(h))
        self._h = h
        if s != LBM_OK:
            msg = L.lbm_batch_last_error(h).decode() if h.value else ""
            if h.value:
                L.lbm_batch_destroy(h)
            self._h = None
            raise LbmError(s, msg)

    def _check(self, s):
        if s != LBM_OK:
            raise LbmError(s, load_library().lbm_batch_last_error(self._h).decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                load_library().lbm_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def close(self):
        self.__del__()

    def step(self, n=1):
        self._check(load_library().lbm_batch_step(self._h, int(n)))

    def tune(self, reps=10):
        """Runs the autotuner; returns the tried shapes (dicts with fluid_ms)."""
        out = (LbmBatchShape * 128)()
        n = C.c_int32()
        self._check(load_library().lbm_batch_tune(self._h, int(reps), out, 128, C.byref(n)))
        return [out[k].as_dict() for k in range(min(n.value, 128))]

    def shape(self):
        sh = LbmBatchShape()
        self._check(load_library().lbm_batch_get_shape(self._h, C.byref(sh)))
        return sh.as_dict()

    def set_shape(self, bulk_v, block, mode=0, per_xcd=0):
        sh = LbmBatchShape(int(bulk_v), int(block), int(mode), int(per_xcd), 0.0)
        self._check(load_library().lbm_batch_set_shape(self._h, C.byref(sh)))

    def time_fluid(self, reps=10):
        ms = C.c_double()
        self._check(load_library().lbm_batch_time_fluid(self._h, int(reps), C.byref(ms)))
        return ms.value

    def set_graph(self, enable):
        self._check(load_library().lbm_batch_set_graph(self._h, int(bool(enable))))


def from_workload(w, precision=None, with_bodies=True):
    lat = Lattice(w.domain, w.tau, w.u_max, precision or w.precision)
    if with_bodies:
        for b in w.bodies:
            lat.add_body(b)
    return lat


_TRAJECTORY = None


def _trajectory_class():
    global _TRAJECTORY
    if _TRAJECTORY is None:
        import torch

        class Trajectory(torch.autograd.Function):
            """J(f0, p) = <lam, g^n> + sum_{t=1..n} <w, g^t> + taylor_weight
            sum_t D_T over n steps of a lattice started from the populations
            f0 (its bodies from their current state), with p = (inlet scale,
            membrane-stiffness scale).  The forward pass runs the lattice's
            discrete adjoint sweep once (lbm_adjoint_run: J from the
            recomputed trajectory, and every derivative); the backward pass
            scales the derivatives by the incoming gradient."""

            @staticmethod
            def forward(ctx, f0, params, lat, n_steps, w, lam, checkpoint_every, taylor_weight, taylor_body):
                if params is not None:
                    lat.set_scales(float(params[0]), float(params[1]))
                lat.set_populations(f0)
                g0, grad, _, J = lat.adjoint_run(n_steps, lam, w, taylor_weight, taylor_body, checkpoint_every)
                ctx.g0, ctx.grad, ctx.has_p = g0, grad, params is not None
                ctx.inlet, ctx.stiff = (float(params[0]), float(params[1])) if params is not None else (1.0, 1.0)
                return torch.tensor(J[0] + taylor_weight * J[1], dtype=torch.float64, device=lat.device)

            @staticmethod
            def backward(ctx, gJ):
                dp = None
                if ctx.has_p:
                    # dJ/ds for the inlet scale; dJ/dkappa for the stiffness scale
                    dp = gJ * torch.stack([ctx.grad[0], ctx.grad[5]])
                return gJ * ctx.g0, dp, None, None, None, None, None, None, None

        _TRAJECTORY = Trajectory
    return _TRAJECTORY


def trajectory(lat, f0, n_steps, w=None, lam=None, checkpoint_every=100, params=None, taylor_weight=0.0,
               taylor_body=0):
    """Differentiable J(f0, params) = <lam, g^n> + sum_{t=1..n} <w, g^t> +
    taylor_weight * sum_t D_T(body taylor_body) over n_steps steps of lat from
    the populations f0 ([19][N] FP64 on the lattice's device; g = f - w_i);
    params (optional, FP64 tensor of 2): the inlet-velocity scale and the
    membrane-stiffness scale (lbm_set_scales), else the lattice's current
    scales.  J.backward() gives dJ/df0 and dJ/dparams through the discrete
    adjoint (lbm_adjoint_run; soft bodies, at most one).  The lattice is left
    holding f0 (the sweep does not step it), at the scales params."""
    return _trajectory_class().apply(f0, params, lat, int(n_steps), w, lam, int(checkpoint_every),
                                     float(taylor_weight), int(taylor_body))
