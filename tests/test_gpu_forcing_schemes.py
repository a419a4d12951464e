"""The two forcing schemes (§2 step 3's velocity shift and Guo's) on flows
with closed-form answers, GPU against the FP64 oracle through the C
interface: a body-force channel between halfway bounce-back walls and a
pressure-balanced periodic force.  The accuracy of each scheme against the
closed form is pinned on the oracle (CPU tests); here the GPU runs must
reproduce the oracle's runs."""
import numpy as np
import pytest

import oracle as O
from gpu_common import make_sim, oracle_params, rel_linf, to_np

pytestmark = pytest.mark.gpu

SCHEMES = {"guo": 0, "shift": 1}


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1904_02108_amd import lbmibm
    return lbmibm


@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_channel(L, scheme):
    """4 x 16 x 4, walls on y, g = 1e-5 along x, tau 0.7: 3000 steps from
    rest (most of the way to the steady parabola) on both sides."""
    shape, tau, g, steps = (4, 16, 4), 0.7, 1e-5, 3000
    fc = SCHEMES[scheme]
    sim = make_sim(L, shape, tau, bc=(0, 1, 0), forcing=fc, g_ext=(g, 0.0, 0.0))
    p = oracle_params(shape, tau, bc=(0, 1, 0), forcing=fc, g_ext=(g, 0.0, 0.0))
    f = O.init_equilibrium(p)
    sim.step(steps)
    O.run(p, f, None, 0, steps)
    rho_r, U_r = O.moments(p, f)
    out = sim.read("rho", "vel")
    e_u = rel_linf(to_np(out["vel"]), U_r)
    d_r = float(np.abs(to_np(out["rho"]) - rho_r).max())  # rho stays 1 up to rounding
    print(scheme, "channel after", steps, "steps: velocity", e_u, "max |d rho|", d_r, flush=True)
    assert e_u < 1e-4 and d_r < 1e-6
    nu = (tau - 0.5) / 3
    y = np.arange(shape[1])
    ref = g / (2 * nu) * (y + 0.5) * (shape[1] - 0.5 - y)
    u = to_np(out["vel"])[0, :, :, :].mean(axis=(0, 2)) + g / 2
    assert np.abs(u - ref).max() / ref.max() < 0.2  # still approaching the steady state


@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_pressure_balanced_force(L, scheme):
    """32 x 4 x 4 periodic with a prescribed G_x = g sin(2 pi x / 32),
    g = 1e-4, tau 0.8: 3000 steps from rest on both sides."""
    shape, tau, g, steps = (32, 4, 4), 0.8, 1e-4, 3000
    fc = SCHEMES[scheme]
    x = np.arange(shape[0])
    G = np.zeros((3,) + shape[::-1])
    G[0] = (g * np.sin(2 * np.pi * x / shape[0]))[None, None, :]
    sim = make_sim(L, shape, tau, forcing=fc)
    sim.write(force=G.astype(np.float32))
    p = oracle_params(shape, tau, forcing=fc)
    f = O.init_equilibrium(p)
    G32 = G.astype(np.float32).astype(np.float64)
    for _ in range(steps):
        f = O.collide_stream(p, f, G32)
    sim.step(steps)
    rho_r, U_r = O.moments(p, f)
    out = sim.read("rho", "vel")
    e_r = rel_linf(to_np(out["rho"]) - 1, rho_r - 1)
    u_phys = to_np(out["vel"]) + G32 / 2
    print(scheme, "pressure-balanced after", steps, "steps: density", e_r,
          "max |U + G/2| / g", np.abs(u_phys).max() / g, flush=True)
    assert e_r < 1e-4
    assert np.abs(u_phys).max() < 1e-3 * g
