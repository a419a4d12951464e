"""Learned warm start of the multi-direct forcing: device-side training data,
training and evaluation helpers over the C interface.

Every arithmetic step runs in the library's kernels (``mlp_train``,
``mlp_forward``, ``mlp_loss_grad``, the feature and warm-start kernels of the
forcing); this module only allocates device memory, slices it and sequences
the calls.
"""
from __future__ import annotations

import numpy as np

from . import lbmibm as L

NPARAM, NFEAT = L.IBM_MLP_NPARAM, L.IBM_MLP_NFEAT


class Network:
    """Parameters and Adam moments of the warm-start MLP in device memory."""

    def __init__(self, theta0, device="cuda", max_batch=4096):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        th = np.ascontiguousarray(theta0, dtype=np.float32).reshape(-1)
        assert th.size == NPARAM
        self.theta = torch.as_tensor(th, device=self.device).clone()
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.t = 0
        self.max_batch = int(max_batch)
        self.ws = torch.empty(L.mlp_workspace_size(self.max_batch), dtype=torch.uint8,
                              device=self.device)

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _workspace(self, batch):
        need = L.mlp_workspace_size(batch)
        if self.ws.numel() < need:
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self.ws

    def train(self, x, t, batch=1024, epochs=1, lr=1e-3):
        """Adam over mini-batches of consecutive rows of x [n,12], t [n,3]
        (device FP32, contiguous); returns the mean batch loss per epoch."""
        assert x.is_contiguous() and t.is_contiguous() and x.shape[0] == t.shape[0]
        ws = self._workspace(batch)
        self.t, losses = L.mlp_train(self.theta.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                     self.t, x.shape[0], x.data_ptr(), t.data_ptr(), batch, epochs,
                                     lr, ws.data_ptr(), self._stream())
        return losses

    def forward(self, x, precision=L.MLP_FP32):
        y = self.torch.empty((x.shape[0], 3), dtype=self.torch.float32, device=self.device)
        L.mlp_forward(self.theta.data_ptr(), x.shape[0], x.data_ptr(), y.data_ptr(), precision,
                      self._workspace(1).data_ptr(), self._stream())
        return y

    def loss_grad(self, x, t):
        torch = self.torch
        g = torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        ws = self._workspace(x.shape[0])
        L.mlp_loss_grad(self.theta.data_ptr(), x.shape[0], x.data_ptr(), t.data_ptr(),
                        g.data_ptr(), loss.data_ptr(), ws.data_ptr(), self._stream())
        return loss, g

    def numpy(self):
        return self.theta.detach().cpu().numpy()


def surface_sim(wl, flags, n_iter, eps=0.0, theta=None, device="cuda"):
    """A simulation of workload ``wl`` with its surface set (FP32 storage)."""
    sim = L.Simulation(wl.shape, wl.tau, bc=wl.bc, forcing=wl.forcing, max_points=wl.n_points,
                       max_iter=max(n_iter, 8), device=device)
    if theta is not None:
        sim.set_mlp(theta)
    sim.set_points(wl.rest, wl.area, wl.body_off, wl.bodies, n_iter, flags, eps)
    return sim


def collect_pairs(wl, n_steps, n_iter=10, skip=0, flags=0, eps=0.0, device="cuda", limit=50.0,
                  stride=1):
    """Training pairs from a plain run of ``wl``: the first-sweep features
    and the final correction of n_steps steps, the first after ``skip``
    warm-up steps and then every ``stride``-th step.
    Returns device tensors x [m,12], t [m,3] with m = n_points * (steps
    kept).  Features and targets are velocities over the body's reference
    speed, of order one while the flow is sound; a run keeps only the steps
    before the first one with a value that is not finite or exceeds
    ``limit`` in magnitude (a diverging flow)."""
    import torch
    sim = surface_sim(wl, flags | L.IBM_KEEP_FEATURES, n_iter, eps, device=device)
    n = wl.n_points
    x = torch.empty((n_steps * n, NFEAT), dtype=torch.float32, device=device)
    t = torch.empty((n_steps * n, 3), dtype=torch.float32, device=device)
    if skip:
        sim.step(skip)
    for k in range(n_steps):
        if k and stride > 1:
            sim.step(stride - 1)
        sim.step(1)
        sim.log_pairs(x[k * n:(k + 1) * n], t[k * n:(k + 1) * n])
    torch.cuda.synchronize(device)
    sim.close()
    xv, tv = x.view(n_steps, -1), t.view(n_steps, -1)
    ok = (torch.isfinite(xv).all(dim=1) & torch.isfinite(tv).all(dim=1) &
          (xv.abs().amax(dim=1) <= limit) & (tv.abs().amax(dim=1) <= limit)).cpu().numpy()
    good = int(np.argmin(ok)) if not ok.all() else n_steps
    return x[:good * n], t[:good * n]


def residual_history(sim, n_steps):
    """Per step: sweeps run and R_rel of every sweep (host sync per step)."""
    out = []
    for _ in range(n_steps):
        sim.step(1)
        st = sim.last_stats()
        den = st["sum_s_ub2"]
        rr = np.sqrt(st["resid"] / den) if den > 0 else np.zeros_like(st["resid"])
        out.append((st["n_iter"], rr))
    return out
