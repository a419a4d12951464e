"""Thin ctypes binding of ``liblbmibm.so`` (C ABI in ``include/lbmibm.h``).

The functions carry the C names and only marshal arguments; every step of the
computation runs in the library's HIP kernels.  ``Simulation`` is a small
convenience owner: it allocates the caller buffers as torch tensors on the
current CUDA (HIP) device, passes torch's current stream, and wraps field
reads/writes into tensors.

Importing this module loads the library and raises ImportError if it has not
been built (``python -m paper_1904_02108_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmibm.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("liblbmibm.so is not built; run `python -m paper_1904_02108_amd.build`")
_lib = ct.CDLL(LIB_PATH)

# enums (mirroring include/lbmibm.h)
LBM_OK, LBM_ERR_ARG, LBM_ERR_OOM, LBM_ERR_HIP, LBM_ERR_STATE, LBM_ERR_DOMAIN, LBM_ERR_NONFINITE = (
    0, -1, -2, -3, -4, -5, -6)
LBM_BC_PERIODIC, LBM_BC_BOUNCEBACK = 0, 1
LBM_STORE_F32, LBM_STORE_F16, LBM_STORE_BF16 = 0, 1, 2
LBM_FORCE_GUO, LBM_FORCE_SHIFT = 0, 1
LBM_NBUF = 5
IBM_INNER_UNWEIGHTED, IBM_STOP_RESIDUAL, IBM_WARM_START, IBM_KEEP_FEATURES, IBM_MLP_FP32 = (
    1, 2, 4, 8, 16)
IBM_WARM_PREV, IBM_U_BOX, IBM_U_KERNEL = 32, 64, 128
MLP_FP32, MLP_BF16 = 0, 1
IBM_MLP_NPARAM, IBM_MLP_NFEAT, IBM_MLP_NNBR = 9347, 12, 16
LBM_MAX_ITER = 64
MLP_NOALLOC_MAX_BATCH = 1024
(LBM_F_RHO, LBM_F_VEL, LBM_F_FORCE, LBM_F_POPS, LBM_F_PT_X, LBM_F_PT_UB, LBM_F_PT_G, LBM_F_PT_DU,
 LBM_F_SUMS, LBM_F_STEP) = (1 << k for k in range(10))

ABI_FUNCTIONS = ("lbm_buffer_sizes", "lbm_create", "lbm_destroy", "lbm_last_error",
                 "ibm_set_points", "ibm_force_iterate", "lbm_step", "lbm_read_fields",
                 "lbm_write_fields", "lbm_set_timing", "lbm_get_timing", "ibm_set_mlp",
                 "ibm_log_pairs", "ibm_last_stats", "mlp_workspace_size", "mlp_forward",
                 "mlp_loss_grad", "mlp_train", "lbm_set_check", "mlp_loss_grad_noalloc")


class lbm_params(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("bc", ct.c_int32 * 3), ("storage", ct.c_int32), ("forcing", ct.c_int32),
                ("tau", ct.c_double), ("rho_wall", ct.c_double), ("wall_u", ct.c_double * 18),
                ("g_ext", ct.c_double * 3), ("rho0", ct.c_double), ("u0", ct.c_double * 3),
                ("max_points", ct.c_int64), ("max_iter", ct.c_int32), ("reserved_", ct.c_int32),
                ("stream", ct.c_void_p)]


class ibm_body(ct.Structure):
    _fields_ = [("center", ct.c_double * 3), ("axis", ct.c_double * 3),
                ("theta0", ct.c_double), ("omega", ct.c_double)]


class ibm_stats(ct.Structure):
    _fields_ = [("n_iter", ct.c_int32), ("pad_", ct.c_int32), ("sum_s", ct.c_double),
                ("sum_s_ub2", ct.c_double), ("resid", ct.c_double * LBM_MAX_ITER)]


class lbm_fields(ct.Structure):
    _fields_ = [("on_device", ct.c_int32), ("pops_f64", ct.c_int32),
                ("rho", ct.c_void_p), ("vel", ct.c_void_p), ("force", ct.c_void_p),
                ("pops", ct.c_void_p), ("pt_x", ct.c_void_p), ("pt_ub", ct.c_void_p),
                ("pt_g", ct.c_void_p), ("pt_du", ct.c_void_p), ("sums", ct.c_void_p),
                ("step", ct.c_void_p)]


_P = ct.POINTER(lbm_params)
_C = ct.c_void_p
_lib.lbm_buffer_sizes.argtypes = [_P, ct.POINTER(ct.c_size_t)]
_lib.lbm_create.argtypes = [_P, ct.POINTER(ct.c_void_p), ct.POINTER(ct.c_void_p)]
_lib.lbm_destroy.argtypes = [_C]
_lib.lbm_destroy.restype = None
_lib.lbm_last_error.argtypes = [_C]
_lib.lbm_last_error.restype = ct.c_char_p
_lib.ibm_set_points.argtypes = [_C, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32,
                                ct.POINTER(ibm_body), ct.c_int32, ct.c_uint32, ct.c_float]
_lib.ibm_force_iterate.argtypes = [_C, ct.POINTER(ibm_stats)]
_lib.lbm_step.argtypes = [_C, ct.c_int32]
_lib.lbm_read_fields.argtypes = [_C, ct.c_uint32, ct.POINTER(lbm_fields)]
_lib.lbm_write_fields.argtypes = [_C, ct.c_uint32, ct.POINTER(lbm_fields)]
_lib.lbm_set_timing.argtypes = [_C, ct.c_int32]
_lib.lbm_set_check.argtypes = [_C, ct.c_int32]
_lib.lbm_get_timing.argtypes = [_C, ct.POINTER(ct.c_double)]
_lib.ibm_set_mlp.argtypes = [_C, ct.c_void_p]
_lib.ibm_log_pairs.argtypes = [_C, ct.c_void_p, ct.c_void_p]
_lib.ibm_last_stats.argtypes = [_C, ct.POINTER(ibm_stats)]
_lib.mlp_workspace_size.argtypes = [ct.c_int64]
_lib.mlp_workspace_size.restype = ct.c_size_t
_lib.mlp_forward.argtypes = [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_int32,
                             ct.c_void_p, ct.c_void_p]
_lib.mlp_loss_grad.argtypes = [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                               ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.mlp_loss_grad_noalloc.argtypes = [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p,
                                       ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.mlp_train.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_int64),
                           ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32,
                           ct.c_double, ct.c_void_p, ct.c_void_p, ct.c_void_p]
for _f in ("lbm_buffer_sizes", "lbm_create", "ibm_set_points", "ibm_force_iterate", "lbm_step",
           "lbm_read_fields", "lbm_write_fields", "lbm_set_timing", "lbm_get_timing",
           "lbm_set_check"):
    getattr(_lib, _f).restype = ct.c_int32


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lbmibm status %d: %s" % (status, msg))
        self.status = status


def lbm_last_error(ctx=None) -> str:
    m = _lib.lbm_last_error(ctx)
    return m.decode() if m else ""


def _check(st, ctx=None):
    if st != LBM_OK:
        raise LbmError(st, lbm_last_error(ctx))


def make_params(shape, tau, bc=(0, 0, 0), storage=LBM_STORE_F32, forcing=LBM_FORCE_GUO,
                rho_wall=1.0, wall_u=None, g_ext=(0.0, 0.0, 0.0), rho0=1.0, u0=(0.0, 0.0, 0.0),
                max_points=0, max_iter=8, stream=None) -> lbm_params:
    p = lbm_params()
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    for a in range(3):
        p.bc[a] = int(bc[a])
    p.storage, p.forcing = int(storage), int(forcing)
    p.tau, p.rho_wall, p.rho0 = float(tau), float(rho_wall), float(rho0)
    wu = np.zeros(18) if wall_u is None else np.asarray(wall_u, dtype=np.float64).reshape(18)
    for k in range(18):
        p.wall_u[k] = float(wu[k])
    for a in range(3):
        p.g_ext[a] = float(g_ext[a])
        p.u0[a] = float(u0[a])
    p.max_points, p.max_iter, p.reserved_ = int(max_points), int(max_iter), 0
    p.stream = stream
    return p


def lbm_buffer_sizes(params: lbm_params):
    sizes = (ct.c_size_t * LBM_NBUF)()
    _check(_lib.lbm_buffer_sizes(ct.byref(params), sizes))
    return [int(s) for s in sizes]


def lbm_create(params: lbm_params, buf_ptrs):
    arr = (ct.c_void_p * LBM_NBUF)(*[int(b) for b in buf_ptrs])
    ctx = ct.c_void_p()
    _check(_lib.lbm_create(ct.byref(params), arr, ct.byref(ctx)))
    return ctx


def lbm_destroy(ctx):
    _lib.lbm_destroy(ctx)


def ibm_set_points(ctx, rest, area, body_off, bodies, n_iter=5, flags=0, eps=0.0):
    rest = np.ascontiguousarray(rest, dtype=np.float32).reshape(-1, 3)
    area = np.ascontiguousarray(area, dtype=np.float32).reshape(-1)
    body_off = np.ascontiguousarray(body_off, dtype=np.int64)
    bodies = np.asarray(bodies, dtype=np.float64).reshape(-1, 8)
    nb = bodies.shape[0]
    btab = (ibm_body * max(nb, 1))()
    for b in range(nb):
        for a in range(3):
            btab[b].center[a] = bodies[b, a]
            btab[b].axis[a] = bodies[b, 3 + a]
        btab[b].theta0, btab[b].omega = bodies[b, 6], bodies[b, 7]
    vp = lambda a: a.ctypes.data_as(ct.c_void_p)
    _check(_lib.ibm_set_points(ctx, rest.shape[0], vp(rest), vp(area), vp(body_off), nb, btab,
                               int(n_iter), int(flags), float(eps)), ctx)


def _stats_dict(s):
    return {"n_iter": s.n_iter, "sum_s": s.sum_s, "sum_s_ub2": s.sum_s_ub2,
            "resid": np.array(s.resid[:s.n_iter])}


def ibm_force_iterate(ctx, stats=False):
    if stats:
        s = ibm_stats()
        _check(_lib.ibm_force_iterate(ctx, ct.byref(s)), ctx)
        return _stats_dict(s)
    _check(_lib.ibm_force_iterate(ctx, None), ctx)
    return None


def ibm_last_stats(ctx):
    s = ibm_stats()
    _check(_lib.ibm_last_stats(ctx, ct.byref(s)), ctx)
    return _stats_dict(s)


def ibm_set_mlp(ctx, theta):
    th = np.ascontiguousarray(theta, dtype=np.float32).reshape(-1)
    if th.size != IBM_MLP_NPARAM:
        raise ValueError("theta must hold %d values" % IBM_MLP_NPARAM)
    _check(_lib.ibm_set_mlp(ctx, th.ctypes.data_as(ct.c_void_p)), ctx)


def ibm_log_pairs(ctx, features_ptr, targets_ptr):
    _check(_lib.ibm_log_pairs(ctx, ct.c_void_p(features_ptr), ct.c_void_p(targets_ptr)), ctx)


def mlp_workspace_size(batch):
    return int(_lib.mlp_workspace_size(int(batch)))


def mlp_forward(theta_ptr, n, x_ptr, y_ptr, precision, workspace_ptr, stream_ptr):
    _check(_lib.mlp_forward(ct.c_void_p(theta_ptr), int(n), ct.c_void_p(x_ptr), ct.c_void_p(y_ptr),
                            int(precision), ct.c_void_p(workspace_ptr), ct.c_void_p(stream_ptr)))


def mlp_loss_grad(theta_ptr, n, x_ptr, t_ptr, grad_ptr, loss_ptr, workspace_ptr, stream_ptr):
    _check(_lib.mlp_loss_grad(ct.c_void_p(theta_ptr), int(n), ct.c_void_p(x_ptr),
                              ct.c_void_p(t_ptr), ct.c_void_p(grad_ptr), ct.c_void_p(loss_ptr),
                              ct.c_void_p(workspace_ptr), ct.c_void_p(stream_ptr)))


def mlp_loss_grad_noalloc(theta_ptr, n, x_ptr, t_ptr, grad_ptr, loss_ptr, stream_ptr):
    _check(_lib.mlp_loss_grad_noalloc(ct.c_void_p(theta_ptr), int(n), ct.c_void_p(x_ptr),
                                      ct.c_void_p(t_ptr), ct.c_void_p(grad_ptr),
                                      ct.c_void_p(loss_ptr), ct.c_void_p(stream_ptr)))


def mlp_train(theta_ptr, m_ptr, v_ptr, step_t, n, x_ptr, t_ptr, batch, n_epochs, lr,
              workspace_ptr, stream_ptr, want_loss=True):
    """Returns (new Adam step count, per-epoch mean batch losses or None)."""
    st = ct.c_int64(int(step_t))
    losses = (ct.c_double * max(int(n_epochs), 1))() if want_loss else None
    _check(_lib.mlp_train(ct.c_void_p(theta_ptr), ct.c_void_p(m_ptr), ct.c_void_p(v_ptr),
                          ct.byref(st), int(n), ct.c_void_p(x_ptr), ct.c_void_p(t_ptr), int(batch),
                          int(n_epochs), float(lr), losses, ct.c_void_p(workspace_ptr),
                          ct.c_void_p(stream_ptr)))
    return st.value, (np.array(losses[:int(n_epochs)]) if want_loss else None)


def lbm_step(ctx, n_steps=1):
    _check(_lib.lbm_step(ctx, int(n_steps)), ctx)


def lbm_read_fields(ctx, mask, fields: lbm_fields):
    _check(_lib.lbm_read_fields(ctx, int(mask), ct.byref(fields)), ctx)


def lbm_write_fields(ctx, mask, fields: lbm_fields):
    _check(_lib.lbm_write_fields(ctx, int(mask), ct.byref(fields)), ctx)


def lbm_set_timing(ctx, enable):
    _check(_lib.lbm_set_timing(ctx, int(enable)), ctx)


def lbm_set_check(ctx, every):
    _check(_lib.lbm_set_check(ctx, int(every)), ctx)


def lbm_get_timing(ctx):
    out = (ct.c_double * 4)()
    _check(_lib.lbm_get_timing(ctx, out), ctx)
    return {"ms_forcing": out[0], "ms_fluid": out[1], "n_forcing": int(out[2]), "n_fluid": int(out[3])}


class Simulation:
    """Owns the caller buffers (torch tensors on ``device``) and one context."""

    def __init__(self, shape, tau, bc=(0, 0, 0), storage=LBM_STORE_F32, forcing=LBM_FORCE_GUO,
                 max_points=0, max_iter=8, device="cuda", **kw):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.shape = tuple(int(v) for v in shape)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            self.params = make_params(shape, tau, bc, storage, forcing, max_points=max_points,
                                      max_iter=max_iter, stream=ct.c_void_p(stream.cuda_stream), **kw)
            sizes = lbm_buffer_sizes(self.params)
            self.bufs = [torch.empty(max(s, 256), dtype=torch.uint8, device=self.device) for s in sizes]
            self.ctx = lbm_create(self.params, [b.data_ptr() for b in self.bufs])
        self.n_points = 0

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncell(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    def grid(self):
        nx, ny, nz = self.shape
        return (nz, ny, nx)

    def set_points(self, rest, area, body_off, bodies, n_iter=5, flags=0, eps=0.0):
        ibm_set_points(self.ctx, rest, area, body_off, bodies, n_iter, flags, eps)
        self.n_points = int(np.asarray(rest).reshape(-1, 3).shape[0])

    def set_check(self, every=1):
        lbm_set_check(self.ctx, every)

    def force_iterate(self, stats=False):
        return ibm_force_iterate(self.ctx, stats)

    def last_stats(self):
        return ibm_last_stats(self.ctx)

    def set_mlp(self, theta):
        ibm_set_mlp(self.ctx, theta)

    def log_pairs(self, features=None, targets=None):
        """Training pairs of the last forcing as device tensors [n, 12] and
        [n, 3] (written into ``features``/``targets`` when given)."""
        t = self.torch
        n = self.n_points
        if features is None:
            features = t.empty((n, IBM_MLP_NFEAT), dtype=t.float32, device=self.device)
        if targets is None:
            targets = t.empty((n, 3), dtype=t.float32, device=self.device)
        assert features.is_contiguous() and targets.is_contiguous()
        assert features.numel() >= n * IBM_MLP_NFEAT and targets.numel() >= n * 3
        ibm_log_pairs(self.ctx, features.data_ptr(), targets.data_ptr())
        return features, targets

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def read(self, *names, pops_f64=False):
        """Returns a dict of torch tensors on the device for the named fields:
        rho, vel, force, pops, pt_x, pt_ub, pt_g, pt_du, sums, step."""
        t = self.torch
        g = self.grid()
        n = self.n_points
        f = lbm_fields()
        f.on_device = 1
        f.pops_f64 = int(pops_f64)
        out, mask = {}, 0
        spec = {"rho": (LBM_F_RHO, g, t.float32), "vel": (LBM_F_VEL, (3,) + g, t.float32),
                "force": (LBM_F_FORCE, (3,) + g, t.float32),
                "pops": (LBM_F_POPS, (19,) + g, t.float64 if pops_f64 else t.float32),
                "pt_x": (LBM_F_PT_X, (n, 3), t.float64), "pt_ub": (LBM_F_PT_UB, (n, 3), t.float32),
                "pt_g": (LBM_F_PT_G, (n, 3), t.float32), "pt_du": (LBM_F_PT_DU, (n, 3), t.float32),
                "sums": (LBM_F_SUMS, (4,), t.float64), "step": (LBM_F_STEP, (1,), t.int64)}
        for name in names:
            bit, shp, dt = spec[name]
            out[name] = t.empty(shp, dtype=dt, device=self.device)
            setattr(f, name, ct.c_void_p(out[name].data_ptr()))
            mask |= bit
        lbm_read_fields(self.ctx, mask, f)
        return out

    def write(self, pops=None, force=None, step=None):
        t = self.torch
        f = lbm_fields()
        f.on_device = 1
        mask, keep = 0, []
        if pops is not None:
            pt = t.as_tensor(pops, device=self.device).contiguous()
            assert pt.dtype in (t.float32, t.float64) and pt.numel() == 19 * self.ncell
            f.pops_f64 = int(pt.dtype == t.float64)
            f.pops = ct.c_void_p(pt.data_ptr())
            keep.append(pt)
            mask |= LBM_F_POPS
        if force is not None:
            ft = t.as_tensor(force, dtype=t.float32, device=self.device).contiguous()
            assert ft.numel() == 3 * self.ncell
            f.force = ct.c_void_p(ft.data_ptr())
            keep.append(ft)
            mask |= LBM_F_FORCE
        if step is not None:
            st = t.tensor([int(step)], dtype=t.int64, device=self.device)
            f.step = ct.c_void_p(st.data_ptr())
            keep.append(st)
            mask |= LBM_F_STEP
        lbm_write_fields(self.ctx, mask, f)
        t.cuda.current_stream(self.device).synchronize()  # keep sources alive until consumed
