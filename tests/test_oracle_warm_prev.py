"""Pins of the oracle's warm start from the previous forcing (flag 32), the
non-learned baseline of the learned warm start: the closed form on a
lattice-aligned plane, the shift identity of the sweep sequence, the
sweep-0 stop and the carry of du from one step to the next.  CPU only."""
import numpy as np
import pytest

import oracle as O

STOP, PREV = 2, 32


def _plane(shape, off, h=1.0):
    nx, ny, nz = shape
    ii, jj = np.meshgrid(np.arange(0, nx, h), np.arange(0, ny, h), indexing="ij")
    return np.stack([ii.ravel() + off[0], jj.ravel() + off[1], np.full(ii.size, off[2])], -1)


@pytest.mark.parametrize("c", [0.0, 1.0, 8.0 / 3.0, 4.0])
def test_warm_prev_on_plane(c):
    """On the lattice-aligned unit-spacing plane (s = 1, U0 = 0) the
    interpolation of a spread constant v is 3/8 v.  Starting from
    du_prev = c u_b: g_1 = (1 - 3c/8) u_b, g_n = (5/8)^(n-1) g_1 and
    du_J = [c + (1 - 3c/8) sum_{n<J-1} (5/8)^n] u_b; c = 8/3 is the fixed
    point (g_n = 0 for n >= 1)."""
    shape = (6, 5, 8)
    p = O.params(shape, 0.7)
    x = _plane(shape, (0.0, 0.0, 3.3))
    ub = np.tile([0.01, 0.02, -0.03], (len(x), 1))
    U0 = np.zeros((3,) + shape[::-1])
    J = 5
    r = O.ibm_ex(p, x, ub, np.ones(len(x)), U0, n_iter=J, flags=PREV, du_prev=c * ub)
    a1 = 1.0 - 3.0 * c / 8.0
    np.testing.assert_allclose(r["du"], ub * (c + a1 * sum((5 / 8) ** n for n in range(J - 1))),
                               rtol=1e-12, atol=1e-17)
    r0 = (ub ** 2).sum()
    want = [r0] + [r0 * a1 ** 2 * (5 / 8) ** (2 * (n - 1)) for n in range(1, J)]
    np.testing.assert_allclose(r["resid"], want, rtol=1e-11, atol=1e-20)
    # the first deficit is that of the untouched field
    assert r["resid"][0] == pytest.approx(r0, rel=1e-14)


def _cloud(seed, shape=(10, 9, 8), n=24):
    rng = np.random.default_rng(seed)
    p = O.params(shape, 0.8)
    x = rng.uniform([2, 2, 2], [shape[0] - 3, shape[1] - 3, shape[2] - 3], size=(n, 3))
    ub = rng.normal(scale=0.02, size=(n, 3))
    s = rng.uniform(0.4, 1.0, n)
    U0 = rng.normal(scale=0.01, size=(3,) + shape[::-1])
    return p, x, ub, s, U0


@pytest.mark.parametrize("K,J", [(1, 2), (3, 3), (2, 5)])
def test_warm_prev_shift_identity(K, J):
    """Starting from the du of K plain sweeps is the same as having run
    them: after its first (interpolation-only) sweep, a J-sweep forcing
    from du_prev = du_K continues the plain sequence, so it equals the
    plain forcing of K + J - 1 sweeps (du, G, last deficit, and residuals
    from sweep K on)."""
    p, x, ub, s, U0 = _cloud(5 + K)
    prev = O.ibm_ex(p, x, ub, s, U0, n_iter=K)
    warm = O.ibm_ex(p, x, ub, s, U0, n_iter=J, flags=PREV, du_prev=prev["du"])
    plain = O.ibm_ex(p, x, ub, s, U0, n_iter=K + J - 1)
    np.testing.assert_allclose(warm["du"], plain["du"], rtol=1e-11, atol=1e-17)
    np.testing.assert_allclose(warm["g"], plain["g"], rtol=1e-10, atol=1e-17)
    np.testing.assert_allclose(warm["G"], plain["G"], rtol=1e-11, atol=1e-18)
    np.testing.assert_allclose(warm["resid"][1:], plain["resid"][K:], rtol=1e-10, atol=1e-24)
    assert warm["resid"][0] == pytest.approx(plain["resid"][0], rel=1e-14)


def test_warm_prev_zero_wastes_one_sweep():
    """du_prev = 0 spreads nothing: the J-sweep forcing equals the plain
    (J - 1)-sweep one with its residuals shifted by one sweep."""
    p, x, ub, s, U0 = _cloud(11)
    J = 4
    warm = O.ibm_ex(p, x, ub, s, U0, n_iter=J, flags=PREV, du_prev=np.zeros_like(ub))
    plain = O.ibm_ex(p, x, ub, s, U0, n_iter=J - 1)
    np.testing.assert_allclose(warm["du"], plain["du"], rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(warm["resid"][1:], plain["resid"], rtol=1e-13)
    assert warm["resid"][0] == pytest.approx(plain["resid"][0], rel=1e-14)


def test_warm_prev_ignored_when_first_sweep_converges():
    """A residual stop met by the first deficit applies s g0 alone; the
    previous du never enters.  Without flag 32 (or without a previous du)
    the forcing is the plain one."""
    p, x, ub, s, U0 = _cloud(13)
    junk = np.full_like(ub, 7.0)
    r = O.ibm_ex(p, x, ub, s, U0, n_iter=5, flags=STOP | PREV, eps=1e3, du_prev=junk)
    assert r["n_sweeps"] == 1
    plain1 = O.ibm_ex(p, x, ub, s, U0, n_iter=1)
    np.testing.assert_array_equal(r["du"], plain1["du"])
    off = O.ibm_ex(p, x, ub, s, U0, n_iter=3, du_prev=junk)
    none = O.ibm_ex(p, x, ub, s, U0, n_iter=3, flags=PREV)
    plain3 = O.ibm_ex(p, x, ub, s, U0, n_iter=3)
    # (the oracle's spread adds in parallel: equal up to rounding order)
    np.testing.assert_allclose(off["du"], plain3["du"], rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(none["du"], plain3["du"], rtol=1e-13, atol=1e-18)


def _rotor(n_iter, flags, du_prev=None):
    shape = (16, 14, 12)
    p = O.params(shape, 0.6)
    rng = np.random.default_rng(17)
    m = 40
    ang = np.linspace(0, 2 * np.pi, m, endpoint=False)
    rest = np.stack([3.0 * np.cos(ang), 3.0 * np.sin(ang), rng.uniform(-1, 1, m)], -1)
    body = np.array([[8.0, 7.0, 6.0, 0.2, 0.3, 1.0, 0.1, 0.01]])
    pts = O.Points(rest, np.full(m, 0.7), [0, m], body, n_iter=n_iter, flags=flags,
                   du_prev=du_prev)
    return p, pts


def test_warm_prev_carried_between_steps():
    """Within a run the du of step t is the previous du of step t + 1; the
    first step has none and is the plain one."""
    p, pts = _rotor(3, PREV)
    f_run = O.init_equilibrium(p, 1.0, (0.01, 0.0, 0.0))
    f_man = f_run.copy()
    f_plain = f_run.copy()
    O.run(p, f_run, pts, 0, 3)
    _, plain_pts = _rotor(3, 0)
    r0 = O.step(p, f_plain, plain_pts, 0)
    r_prev = O.step(p, f_man, pts, 0)
    np.testing.assert_allclose(r_prev["du"], r0["du"], rtol=1e-13, atol=1e-18)
    for t in (1, 2):
        _, pts_t = _rotor(3, PREV, du_prev=r_prev["du"])
        r_prev = O.step(p, f_man, pts_t, t)
    np.testing.assert_allclose(f_run, f_man, rtol=0, atol=1e-15)


def test_warm_prev_winds_up_along_a_null_direction():
    """Why the carried correction can diverge where a truncated sweep cannot.
    Two coincident points (s = 1) with opposite velocities +-u: the spread of
    any du with du_1 = -du_2 vanishes, so interpolation keeps returning the
    untouched field (U0 = 0) and the deficit stays g = u_b in every sweep.
    The plain N-sweep forcing ends with du = N u_b, every step afresh; warm
    started from the previous du, the T-th forcing ends with
    du = (N + (T - 1)(N - 1)) u_b, growing without bound while G stays 0 and
    the residual never drops.  Surfaces of neighbouring bodies that cross
    with different velocities have such directions (nearly: their spread is
    small but not zero, so G grows too)."""
    shape = (12, 12, 12)
    p = O.params(shape, 0.7)
    x = np.array([[5.3, 6.1, 4.7], [5.3, 6.1, 4.7]])
    u = np.array([0.02, -0.01, 0.03])
    ub = np.stack([u, -u])
    s = np.ones(2)
    U0 = np.zeros((3,) + shape[::-1])
    N = 4
    plain = O.ibm_ex(p, x, ub, s, U0, n_iter=N)
    np.testing.assert_allclose(plain["du"], N * ub, rtol=1e-14)
    du = None
    for T in range(1, 7):
        r = O.ibm_ex(p, x, ub, s, U0, n_iter=N, flags=PREV if du is not None else 0,
                     du_prev=du)
        du = r["du"]
        np.testing.assert_allclose(du, (N + (T - 1) * (N - 1)) * ub, rtol=1e-13)
        np.testing.assert_allclose(r["resid"], np.full(N, (ub ** 2).sum()), rtol=1e-13)
        assert np.abs(r["G"]).max() < 1e-15
