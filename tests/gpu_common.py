"""Shared helpers of the GPU parity tests: build the HIP simulation and the
oracle from the same seeded inputs and compare fields."""
import numpy as np

import oracle as O


def rel_linf(a, b):
    """max |a - b| / max |b| (b is the oracle's field)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def wrap_diff(a, b, shape, bc):
    """a - b for point positions [n,3], folded on periodic axes."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    for ax in range(3):
        if bc[ax] == 0:
            n = shape[ax]
            d[:, ax] -= n * np.round(d[:, ax] / n)
    return d


def make_sim(L, shape, tau, bc=(0, 0, 0), storage=0, forcing=0, max_points=0, max_iter=8, **kw):
    return L.Simulation(shape, tau, bc=bc, storage=storage, forcing=forcing,
                        max_points=max_points, max_iter=max_iter, **kw)


def oracle_params(shape, tau, bc=(0, 0, 0), forcing=0, wall_u=None, g_ext=(0, 0, 0), rho_wall=1.0):
    return O.params(shape, tau, bc=bc, forcing=forcing, wall_u=wall_u, g_ext=g_ext,
                    rho_wall=rho_wall)


def sim_for_workload(L, wl, storage=0, flags=0, extra_points=0):
    sim = make_sim(L, wl.shape, wl.tau, bc=wl.bc, storage=storage, forcing=wl.forcing,
                   max_points=wl.n_points + extra_points, max_iter=max(wl.n_iter, 8))
    if wl.n_points:
        sim.set_points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter, flags)
    p = oracle_params(wl.shape, wl.tau, bc=wl.bc, forcing=wl.forcing)
    pts = O.Points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter, flags) if wl.n_points else None
    return sim, p, pts


def to_np(t):
    return t.detach().cpu().numpy()
