"""The point layout the forcing kernels rely on, checked on the host for the
benchmark family's surfaces over a full turn of every body (§3: Algorithm 1
moves the points; the 4-point kernel of a point at x reaches the cells
floor(x) - 1 .. floor(x) + 2 on each axis).  Positions come from the
oracle's FP64 kinematics; the base cell and fraction are formed as the
library forms them (the fraction rounded to FP32; one that rounds up to 1
moves the base cell by one).

* Every tap of a point lies in the 11^3 box [o - 1, o + 10) of its owner
  tile (o = 8 floor(base / 8) per axis, base wrapped on periodic axes), so
  the box the sweep stages in LDS holds every U value the point
  interpolates and receives every value it spreads, and the box index of
  any tap (first tap plus an offset of at most 3 per axis) is below 11^3.
* On a walled axis every tap lies inside the lattice, the condition that
  ibm_set_points enforces (LBM_ERR_DOMAIN) for every rotation angle.
"""
import numpy as np
import pytest

import oracle as O
from paper_1904_02108_amd import workload as W

TILE, BOX = 8, 11


def base_and_frac(x):
    """Base cell and FP32 fraction per coordinate, as the library forms them."""
    fl = np.floor(x)
    base = fl.astype(np.int64)
    frac = (x - fl).astype(np.float32)
    up = frac >= np.float32(1.0)
    base[up] += 1
    frac[up] = 0.0
    return base, frac


def check_layout(wl, steps, sample=None, seed=0):
    rest, body_off, bodies = wl.rest, wl.body_off, wl.bodies
    idx = None
    if sample is not None and wl.n_points > sample:
        idx = np.sort(np.random.default_rng(seed).choice(wl.n_points, sample, replace=False))
    n = np.array(wl.shape)  # (nx, ny, nz), as the positions (x, y, z)
    bc = np.array(wl.bc)
    for s in steps:
        x, _ = O.kinematics(rest, body_off, bodies, s)
        if idx is not None:
            x = x[idx]
        base, frac = base_and_frac(x)
        assert np.all((frac >= 0) & (frac < 1))
        for a in range(3):
            if bc[a] == 0:
                b = np.mod(base[:, a], n[a])
            else:
                b = base[:, a]
                # walled axis: every tap (b - 1 .. b + 2) inside the lattice
                assert b.min() - 1 >= 0 and b.max() + 2 <= n[a] - 1, (wl.name, s, a)
            o = (b // TILE) * TILE
            lo, hi = b - 1 - o, b + 2 - o  # first and last tap, relative to the origin
            assert lo.min() >= -1 and hi.max() <= BOX - 2, (wl.name, s, a)
            # box index of the first tap along this axis, and of the last
            first = lo + 1
            assert first.min() >= 0 and first.max() + 3 <= BOX - 1


def turn_steps(bodies, k=12):
    """k steps spread over a full turn of the slowest body (and step 0, 1)."""
    w = np.abs(np.asarray(bodies)[:, 7])
    w = w[w > 0]
    period = int(np.ceil(2 * np.pi / w.min())) if w.size else 1
    return sorted(set([0, 1] + [int(period * j / k) for j in range(1, k + 1)]))


@pytest.mark.parametrize("name", ["c0", "c1", "c1_dense", "c2", "c2_dense"])
def test_layout_benchmark_configs(name):
    wl = W.config(name)
    check_layout(wl, turn_steps(wl.bodies), sample=40000)


@pytest.mark.parametrize("n_props", [1, 6, 18])
def test_layout_paper_family(n_props):
    wl = W.paper_family(n_props)
    check_layout(wl, turn_steps(wl.bodies), sample=40000)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (0, 1, 1)])
def test_layout_small_box_with_walls(bc):
    wl = W.tiny_propeller_case(bc=bc)
    check_layout(wl, turn_steps(wl.bodies))


def test_box_index_bound_is_tight():
    """The largest first-tap box index plus the largest tap offset is the last
    cell of the box: 11^3 is the smallest box for 8^3 tiles and 4 taps."""
    first_max = (TILE - 1) * (1 + BOX + BOX * BOX)
    last_offset = 3 * (1 + BOX + BOX * BOX)
    assert first_max + last_offset == BOX ** 3 - 1
