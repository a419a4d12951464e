"""Writes c1_500_steps.npz: the FP64 oracle's state of the single-propeller
case C1 (128^3, walls on y and z, one propeller at h 0.7) after 500 steps
from rest, sampled, for the GPU's long-run comparison (FP32 and 16-bit
storage).  Calls only the oracle and the input generator.

Stored (FP32, far finer than the comparison's tolerances): density and
velocity at 2048 seeded cells plus every cell of a 16^3 block that the
blade tips sweep through, the force G of the 500th step at the same cells,
every point's correction du of that step, and the FP64 mass sum.
Run: python tests/golden/make_c1_500.py (a few minutes on 8 cores).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1904_02108_amd import workload as W  # noqa: E402

STEPS = 500


def sample_cells(shape):
    """Seeded sample cells (z, y, x): 2048 uniform ones and a 16^3 block
    that the blade tips sweep through (the propeller of tip radius 52 is
    centred at 64 and turns about z)."""
    rng = np.random.default_rng(500)
    nx, ny, nz = shape
    rnd = np.stack([rng.integers(0, nz, 2048), rng.integers(0, ny, 2048),
                    rng.integers(0, nx, 2048)], -1)
    zz, yy, xx = np.meshgrid(np.arange(56, 72), np.arange(108, 124), np.arange(56, 72),
                             indexing="ij")
    blk = np.stack([zz.ravel(), yy.ravel(), xx.ravel()], -1)
    return np.concatenate([rnd, blk]).astype(np.int16)


def main():
    wl = W.config("c1")
    p = O.params(wl.shape, wl.tau, bc=wl.bc, forcing=wl.forcing)
    pts = O.Points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
    f = O.init_equilibrium(p)
    O.run(p, f, pts, 0, STEPS - 1)
    r = O.step(p, f, pts, STEPS - 1)      # step 500's forcing, then its stream-collide
    rho, U = O.moments(p, f)
    cells = sample_cells(wl.shape)
    z, y, x = cells.T.astype(np.int64)
    f32 = np.float32
    np.savez_compressed(
        os.path.join(HERE, "c1_500_steps.npz"),
        steps=np.int64(STEPS), cells=cells, rho_minus_1=(rho[z, y, x] - 1.0).astype(f32),
        vel=U[:, z, y, x].astype(f32), force=r["G"][:, z, y, x].astype(f32),
        du=r["du"].astype(f32), mass=np.float64(O.sums(p, f)[0]))


if __name__ == "__main__":
    main()
