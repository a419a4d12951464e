"""Writes c2_dense_half_200_steps.npz: the FP64 oracle's state of the dense
64-propeller geometry (256^3 periodic, tau 0.55, h 0.41, 1 596 800 points)
with every rotation rate halved, after 200 steps from rest, sampled, for the
GPU's long-run comparison of the three storage formats.  The configured
rates drive this flow unstable within a few tens of steps; at half rates it
stays sound, so errors against the oracle measure the storage and not a
blow-up.  Calls only the oracle and the input generator.

Stored (FP32, far finer than the comparison's tolerances): density and
velocity at 4096 seeded cells plus every cell of a 16^3 block between the
first two propellers, where their blade tips pass each other; the force G
of the 200th step at the same cells; the correction du of that step for
every point of the first propeller and for 8192 seeded points of the
others; and the FP64 mass and momentum sums.
Run: python tests/golden/make_c2_half.py (about half an hour on 8 cores).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1904_02108_amd import workload as W  # noqa: E402

STEPS = 200


def sample_cells(shape):
    """Seeded cells (z, y, x): 4096 uniform ones and the 16^3 block
    x 56..71, y 24..39, z 24..39 between the propellers centred at
    (32, 32, 32) and (96, 32, 32)."""
    rng = np.random.default_rng(200)
    nx, ny, nz = shape
    rnd = np.stack([rng.integers(0, nz, 4096), rng.integers(0, ny, 4096),
                    rng.integers(0, nx, 4096)], -1)
    zz, yy, xx = np.meshgrid(np.arange(24, 40), np.arange(24, 40), np.arange(56, 72),
                             indexing="ij")
    blk = np.stack([zz.ravel(), yy.ravel(), xx.ravel()], -1)
    return np.concatenate([rnd, blk]).astype(np.int16)


def sample_points(body_off):
    """Every point of the first propeller and 8192 seeded points of the rest."""
    rng = np.random.default_rng(201)
    first = np.arange(body_off[0], body_off[1])
    rest = np.sort(rng.choice(np.arange(body_off[1], body_off[-1]), 8192, replace=False))
    return np.concatenate([first, rest]).astype(np.int32)


def main():
    wl = W.config("c2_dense_half")
    p = O.params(wl.shape, wl.tau, bc=wl.bc, forcing=wl.forcing)
    pts = O.Points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
    f = O.init_equilibrium(p)
    t0 = time.time()
    for s0 in range(0, STEPS - 1, 20):
        n = min(20, STEPS - 1 - s0)
        O.run(p, f, pts, s0, n)
        print("steps %d: %.0f s" % (s0 + n, time.time() - t0), flush=True)
    r = O.step(p, f, pts, STEPS - 1)      # step 200's forcing, then its stream-collide
    rho, U = O.moments(p, f)
    sums = O.sums(p, f)
    cells = sample_cells(wl.shape)
    z, y, x = cells.T.astype(np.int64)
    pidx = sample_points(wl.body_off)
    f32 = np.float32
    np.savez_compressed(
        os.path.join(HERE, "c2_dense_half_200_steps.npz"),
        steps=np.int64(STEPS), cells=cells, rho_minus_1=(rho[z, y, x] - 1.0).astype(f32),
        vel=U[:, z, y, x].astype(f32), force=r["G"][:, z, y, x].astype(f32),
        points=pidx, du=r["du"][pidx].astype(f32), sums=sums.astype(np.float64),
        max_abs_velocity=np.float64(np.abs(U).max()), rho_range=np.array([rho.min(), rho.max()]))
    print("done: max|U| %.4f, rho [%.4f, %.4f], mass drift %.3e" % (
        np.abs(U).max(), rho.min(), rho.max(), abs(sums[0] - wl.n_cells) / wl.n_cells), flush=True)


if __name__ == "__main__":
    main()
