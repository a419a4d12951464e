"""ctypes front end of the FP64 oracle (``lbm_ibm_oracle.c``).

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it.  It builds the C source with gcc on first
use (or when the source is newer than the shared library) and exposes numpy
functions whose names follow the C entry points.

Array conventions (shared with the HIP library's export format only by
definition, not by code):
  populations f: float64 [19, nz, ny, nx], D3Q19 order of the C source
  rho: [nz, ny, nx]; U, G: [3, nz, ny, nx]
  points: [n, 3]; bodies: [nb, 8] = (cx, cy, cz, ax, ay, az, theta0, omega)
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_ibm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

BC_PERIODIC, BC_BOUNCEBACK = 0, 1
FORCE_GUO, FORCE_SHIFT = 0, 1
IBM_INNER_UNWEIGHTED = 1
IBM_STOP_RESIDUAL = 2
IBM_WARM_START = 4
IBM_WARM_PREV = 32


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, strict IEEE double)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("bc", ct.c_int32 * 3), ("forcing", ct.c_int32), ("pad_", ct.c_int32),
                ("tau", ct.c_double), ("rho_wall", ct.c_double),
                ("wall_u", ct.c_double * 18), ("g_ext", ct.c_double * 3)]


class _Points(ct.Structure):
    _fields_ = [("npts", ct.c_int64), ("rest", ct.c_void_p), ("area", ct.c_void_p),
                ("body_off", ct.c_void_p), ("nbodies", ct.c_int32), ("n_iter", ct.c_int32),
                ("flags", ct.c_int32), ("pad_", ct.c_int32), ("bodies", ct.c_void_p),
                ("eps", ct.c_double), ("theta", ct.c_void_p), ("du_prev", ct.c_void_p)]


class _IbmOpts(ct.Structure):
    _fields_ = [("n_iter", ct.c_int32), ("flags", ct.c_int32), ("eps", ct.c_double),
                ("theta", ct.c_void_p), ("nbr", ct.c_void_p), ("v_pt", ct.c_void_p),
                ("du_prev", ct.c_void_p)]


class _StepOut(ct.Structure):
    _fields_ = [("sums", ct.c_void_p), ("G", ct.c_void_p), ("x", ct.c_void_p),
                ("ub", ct.c_void_p), ("g", ct.c_void_p), ("du", ct.c_void_p),
                ("resid", ct.c_void_p), ("feat", ct.c_void_p), ("n_sweeps", ct.c_void_p)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ct.CDLL(build())
            P = ct.POINTER(Params)
            vp, i64, i32, d = ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_double
            lib.orc_d3q19.argtypes = [vp, vp, vp]
            lib.orc_equilibrium.argtypes = [d, vp, vp]
            lib.orc_moments.argtypes = [P, vp, vp, vp]
            lib.orc_init_equilibrium.argtypes = [P, d, vp, vp]
            lib.orc_collide_stream.argtypes = [P, vp, vp, vp]
            lib.orc_sums.argtypes = [P, vp, vp]
            lib.orc_delta.argtypes = [d]
            lib.orc_delta.restype = d
            lib.orc_interpolate.argtypes = [P, i64, vp, vp, vp]
            lib.orc_interpolate.restype = ct.c_int
            lib.orc_spread.argtypes = [P, i64, vp, vp, vp]
            lib.orc_spread.restype = ct.c_int
            lib.orc_kinematics.argtypes = [i64, vp, vp, i32, vp, i64, vp, vp]
            lib.orc_ibm.argtypes = [P, i64, vp, vp, vp, vp, ct.POINTER(_IbmOpts), vp, vp, vp,
                                    vp, vp, vp]
            lib.orc_ibm.restype = ct.c_int
            lib.orc_step.argtypes = [P, vp, ct.POINTER(_Points), i64, ct.POINTER(_StepOut)]
            lib.orc_step.restype = ct.c_int
            lib.orc_run.argtypes = [P, vp, ct.POINTER(_Points), i64, i64, vp, vp]
            lib.orc_neighbours.argtypes = [i64, vp, vp, i32, vp, i64, vp]
            lib.orc_vref.argtypes = [vp, vp, i32, vp, vp]
            lib.orc_features.argtypes = [i64, vp, vp, vp, vp, vp]
            lib.orc_run.restype = ct.c_int
            lib.orc_mlp_nparam.restype = ct.c_int32
            lib.orc_mlp_forward.argtypes = [vp, i64, vp, vp]
            lib.orc_mlp_loss_grad.argtypes = [vp, i64, vp, vp, vp]
            lib.orc_mlp_loss_grad.restype = d
            lib.orc_adam_step.argtypes = [vp, vp, vp, vp, i64, d, d, d, d]
            lib.orc_set_threads.argtypes = [ct.c_int]
            lib.orc_set_threads.restype = ct.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError("oracle returned %d (support outside a walled box)" % rc)


def params(shape, tau, bc=(0, 0, 0), forcing=FORCE_GUO, rho_wall=1.0,
           wall_u=None, g_ext=(0.0, 0.0, 0.0)) -> Params:
    """shape = (nx, ny, nz); wall_u[axis][face][component] (face 0 = low)."""
    p = Params()
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    for a in range(3):
        p.bc[a] = int(bc[a])
    p.forcing = int(forcing)
    p.tau = float(tau)
    p.rho_wall = float(rho_wall)
    wu = np.zeros((3, 2, 3)) if wall_u is None else np.asarray(wall_u, dtype=np.float64)
    for i, v in enumerate(wu.reshape(-1)):
        p.wall_u[i] = float(v)
    for a in range(3):
        p.g_ext[a] = float(g_ext[a])
    return p


def grid_shape(p: Params):
    return (p.nz, p.ny, p.nx)


def d3q19():
    lib = _load()
    e = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    lib.orc_d3q19(_ptr(e), _ptr(w), _ptr(opp))
    return e, w, opp


def delta(r):
    lib = _load()
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda v: lib.orc_delta(float(v)), otypes=[np.float64])(r)


def equilibrium(rho, u):
    lib = _load()
    u = _f64(u)
    eq = np.zeros(19)
    lib.orc_equilibrium(float(rho), _ptr(u), _ptr(eq))
    return eq


def init_equilibrium(p, rho0=1.0, u0=(0.0, 0.0, 0.0)):
    lib = _load()
    f = np.zeros((19,) + grid_shape(p))
    u0 = _f64(u0)
    lib.orc_init_equilibrium(ct.byref(p), float(rho0), _ptr(u0), _ptr(f))
    return f


def moments(p, f):
    lib = _load()
    f = _f64(f)
    rho = np.zeros(grid_shape(p))
    U = np.zeros((3,) + grid_shape(p))
    lib.orc_moments(ct.byref(p), _ptr(f), _ptr(rho), _ptr(U))
    return rho, U


def collide_stream(p, f, G=None):
    lib = _load()
    f = _f64(f)
    out = np.zeros_like(f)
    Gc = None if G is None else _f64(G)
    lib.orc_collide_stream(ct.byref(p), _ptr(f), _ptr(Gc), _ptr(out))
    return out


def sums(p, f):
    lib = _load()
    f = _f64(f)
    out = np.zeros(4)
    lib.orc_sums(ct.byref(p), _ptr(f), _ptr(out))
    return out


def interpolate(p, x, U):
    lib = _load()
    x = _f64(x).reshape(-1, 3)
    U = _f64(U)
    u = np.zeros_like(x)
    _check(lib.orc_interpolate(ct.byref(p), x.shape[0], _ptr(x), _ptr(U), _ptr(u)))
    return u


def spread(p, x, v, acc=None):
    lib = _load()
    x = _f64(x).reshape(-1, 3)
    v = _f64(v).reshape(-1, 3)
    acc = np.zeros((3,) + grid_shape(p)) if acc is None else _f64(acc).copy()
    _check(lib.orc_spread(ct.byref(p), x.shape[0], _ptr(x), _ptr(v), _ptr(acc)))
    return acc


def kinematics(rest, body_off, bodies, step):
    lib = _load()
    rest = _f64(rest).reshape(-1, 3)
    body_off = np.ascontiguousarray(body_off, dtype=np.int64)
    bodies = _f64(bodies).reshape(-1, 8)
    x = np.zeros_like(rest)
    ub = np.zeros_like(rest)
    lib.orc_kinematics(rest.shape[0], _ptr(rest), _ptr(body_off), bodies.shape[0],
                       _ptr(bodies), int(step), _ptr(x), _ptr(ub))
    return x, ub


def ibm(p, x, ub, s, U0, n_iter=5, flags=0):
    """Returns G [3,nz,ny,nx], du [n,3], g_last [n,3], resid [n_iter]."""
    r = ibm_ex(p, x, ub, s, U0, n_iter=n_iter, flags=flags)
    return r["G"], r["du"], r["g"], r["resid"]


def ibm_ex(p, x, ub, s, U0, n_iter=5, flags=0, eps=0.0, theta=None, nbr=None, v_pt=None,
           features=False, du_prev=None):
    """Forcing with every option: residual stop (flags 2, eps), warm start
    (flags 4, theta, nbr [n,16] int32, v_pt [n]), warm start from a previous
    correction (flags 32, du_prev [n,3]); features=True also returns
    the features of the first sweep (needs nbr and v_pt).  Returns a dict
    with G, du, g (last sweep), resid [n_sweeps], n_sweeps, feat."""
    lib = _load()
    x = _f64(x).reshape(-1, 3)
    ub = _f64(ub).reshape(-1, 3)
    s = _f64(s).reshape(-1)
    U0 = _f64(U0)
    n = x.shape[0]
    o = _IbmOpts()
    o.n_iter, o.flags, o.eps = int(n_iter), int(flags), float(eps)
    keep = []
    if theta is not None:
        keep.append(_f64(theta))
        o.theta = _ptr(keep[-1])
    if nbr is not None:
        keep.append(np.ascontiguousarray(nbr, dtype=np.int32))
        o.nbr = _ptr(keep[-1])
    if v_pt is not None:
        keep.append(_f64(v_pt))
        o.v_pt = _ptr(keep[-1])
    if du_prev is not None:
        keep.append(_f64(du_prev).reshape(-1, 3))
        o.du_prev = _ptr(keep[-1])
    res = {"G": np.zeros((3,) + grid_shape(p)), "du": np.zeros((n, 3)), "g": np.zeros((n, 3))}
    resid = np.zeros(max(int(n_iter), 1))
    ns = np.zeros(1, dtype=np.int32)
    feat = np.zeros((n, 12)) if features else None
    _check(lib.orc_ibm(ct.byref(p), n, _ptr(x), _ptr(ub), _ptr(s), _ptr(U0), ct.byref(o),
                       _ptr(res["G"]), _ptr(res["du"]), _ptr(res["g"]), _ptr(resid),
                       _ptr(feat), _ptr(ns)))
    res["n_sweeps"] = int(ns[0])
    res["resid"] = resid[:res["n_sweeps"]]
    res["feat"] = feat
    return res


def neighbours(rest, body_off, idx=None):
    """N(k) of the warm-start features: [n,16] int32 (-1 pads); with idx,
    only the listed rows are computed (the others are -2)."""
    lib = _load()
    rest = _f64(rest).reshape(-1, 3)
    body_off = np.ascontiguousarray(body_off, dtype=np.int64)
    nbr = np.full((rest.shape[0], 16), -2, dtype=np.int32)
    if idx is None:
        lib.orc_neighbours(rest.shape[0], _ptr(rest), _ptr(body_off), body_off.size - 1, None, 0,
                           _ptr(nbr))
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        lib.orc_neighbours(rest.shape[0], _ptr(rest), _ptr(body_off), body_off.size - 1,
                           _ptr(idx), idx.size, _ptr(nbr))
    return nbr


def vref(rest, body_off, bodies):
    """Reference speed of each body [nb]."""
    lib = _load()
    rest = _f64(rest).reshape(-1, 3)
    body_off = np.ascontiguousarray(body_off, dtype=np.int64)
    bodies = _f64(bodies).reshape(-1, 8)
    out = np.zeros(bodies.shape[0])
    lib.orc_vref(_ptr(rest), _ptr(body_off), bodies.shape[0], _ptr(bodies), _ptr(out))
    return out


def vref_points(rest, body_off, bodies):
    """Reference speed of each point's body [n]."""
    vb = vref(rest, body_off, bodies)
    body_off = np.asarray(body_off, dtype=np.int64)
    return np.repeat(vb, np.diff(body_off))


def features(g0, ub, nbr, v_pt):
    """Warm-start features [n,12] from the first deficit g0 and u_b [n,3]."""
    lib = _load()
    g0 = _f64(g0).reshape(-1, 3)
    ub = _f64(ub).reshape(-1, 3)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    v_pt = _f64(v_pt).reshape(-1)
    out = np.zeros((g0.shape[0], 12))
    lib.orc_features(g0.shape[0], _ptr(g0), _ptr(ub), _ptr(nbr), _ptr(v_pt), _ptr(out))
    return out


class Points:
    """Lagrangian surface description handed to the step functions."""

    def __init__(self, rest, area, body_off, bodies, n_iter=5, flags=0, eps=0.0, theta=None,
                 du_prev=None):
        self.rest = _f64(rest).reshape(-1, 3)
        self.area = _f64(area).reshape(-1)
        self.body_off = np.ascontiguousarray(body_off, dtype=np.int64)
        self.bodies = _f64(bodies).reshape(-1, 8)
        self.n_iter = int(n_iter)
        self.flags = int(flags)
        self.eps = float(eps)
        self.theta = None if theta is None else _f64(theta).reshape(-1)
        self.du_prev = None if du_prev is None else _f64(du_prev).reshape(-1, 3)
        self.c = _Points(self.rest.shape[0], _ptr(self.rest), _ptr(self.area),
                         _ptr(self.body_off), self.bodies.shape[0], self.n_iter,
                         self.flags, 0, _ptr(self.bodies), self.eps, _ptr(self.theta),
                         _ptr(self.du_prev))

    @property
    def n(self):
        return self.rest.shape[0]


def step(p, f, pts=None, step_index=0, outputs=True, features=False):
    """One full time step in place on f (float64 [19,nz,ny,nx], C-contiguous).

    Returns a dict with sums (before the step), G, x, ub, g, du, resid
    [n_sweeps], n_sweeps, and with features=True feat [n,12]."""
    lib = _load()
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
    o = _StepOut()
    res = {}
    if outputs:
        res["sums"] = np.zeros(4)
        res["G"] = np.zeros((3,) + grid_shape(p))
        o.sums, o.G = _ptr(res["sums"]), _ptr(res["G"])
        if pts is not None and pts.n > 0:
            for k in ("x", "ub", "g", "du"):
                res[k] = np.zeros((pts.n, 3))
            res["resid"] = np.zeros(max(pts.n_iter, 1))
            o.x, o.ub, o.g, o.du = (_ptr(res[k]) for k in ("x", "ub", "g", "du"))
            o.resid = _ptr(res["resid"])
            res["n_sweeps"] = np.zeros(1, dtype=np.int32)
            o.n_sweeps = _ptr(res["n_sweeps"])
            if features:
                res["feat"] = np.zeros((pts.n, 12))
                o.feat = _ptr(res["feat"])
    pc = ct.byref(pts.c) if pts is not None else None
    _check(lib.orc_step(ct.byref(p), _ptr(f), pc, int(step_index), ct.byref(o)))
    if "n_sweeps" in res:
        res["n_sweeps"] = int(res["n_sweeps"][0])
        res["resid"] = res["resid"][:res["n_sweeps"]]
    return res


def run(p, f, pts=None, step0=0, n_steps=1, sweeps=False):
    """n_steps steps in place on f; returns the sums before each step (and,
    with sweeps=True, also the sweeps of each step's forcing)."""
    lib = _load()
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
    hist = np.zeros((int(n_steps), 4))
    sw = np.zeros(int(n_steps), dtype=np.int32)
    pc = ct.byref(pts.c) if pts is not None else None
    _check(lib.orc_run(ct.byref(p), _ptr(f), pc, int(step0), int(n_steps), _ptr(hist), _ptr(sw)))
    return (hist, sw) if sweeps else hist


# ------------------------------------------------------------ learned warm start
def set_threads(n=0):
    """Set the oracle's OpenMP thread count (n > 0); returns the count in effect."""
    return int(_load().orc_set_threads(int(n)))


def mlp_nparam():
    return int(_load().orc_mlp_nparam())


def mlp_forward(theta, x):
    """x: [n, 12] -> y: [n, 3] (FP64)."""
    lib = _load()
    theta = _f64(theta).reshape(-1)
    x = _f64(x).reshape(-1, 12)
    y = np.zeros((x.shape[0], 3))
    lib.orc_mlp_forward(_ptr(theta), x.shape[0], _ptr(x), _ptr(y))
    return y


def mlp_loss_grad(theta, x, t):
    """Mean squared error over samples and outputs and its gradient."""
    lib = _load()
    theta = _f64(theta).reshape(-1)
    x = _f64(x).reshape(-1, 12)
    t = _f64(t).reshape(-1, 3)
    g = np.zeros(mlp_nparam())
    loss = lib.orc_mlp_loss_grad(_ptr(theta), x.shape[0], _ptr(x), _ptr(t), _ptr(g))
    return loss, g


def adam_step(theta, grad, m, v, step_t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on theta, m, v (float64 arrays)."""
    lib = _load()
    for a in (theta, grad, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib.orc_adam_step(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), int(step_t), float(lr),
                      float(beta1), float(beta2), float(eps))
