"""Pins of the oracle's residual-stopped forcing and of the learned warm
start's inputs (neighbour lists, reference speed, features) and its effect
on the sweep: closed forms on a lattice-aligned plane, the matrix form of
the sweep on a tiny grid, and special parameter choices.  CPU only."""
import numpy as np
import pytest

import oracle as O

NP = 9347
STOP, WARM = 2, 4


def _plane(shape, off, h=1.0):
    nx, ny, nz = shape
    ii, jj = np.meshgrid(np.arange(0, nx, h), np.arange(0, ny, h), indexing="ij")
    return np.stack([ii.ravel() + off[0], jj.ravel() + off[1], np.full(ii.size, off[2])], -1)


# ------------------------------------------------------------ residual stop
@pytest.mark.parametrize("k_stop", [0, 1, 3])
def test_residual_stop_on_plane(k_stop):
    """On the lattice-aligned plane g_n = (5/8)^n u_b, so the residual of
    sweep n is (5/8)^(2n) sum s|u_b|^2 and a threshold eps = (5/8)^(k-1/2)
    stops after sweep k, with du = u_b sum_{n<=k} (5/8)^n."""
    shape = (6, 5, 8)
    p = O.params(shape, 0.7)
    x = _plane(shape, (0.0, 0.0, 3.3))
    ub = np.tile([0.01, 0.02, -0.03], (len(x), 1))
    U0 = np.zeros((3,) + shape[::-1])
    eps = (5 / 8) ** (k_stop - 0.5)
    r = O.ibm_ex(p, x, ub, np.ones(len(x)), U0, n_iter=8, flags=STOP, eps=eps)
    assert r["n_sweeps"] == k_stop + 1
    np.testing.assert_allclose(r["du"], ub * sum((5 / 8) ** n for n in range(k_stop + 1)),
                               rtol=1e-12)
    r0 = (ub ** 2).sum()
    np.testing.assert_allclose(r["resid"], [r0 * (5 / 8) ** (2 * n) for n in range(k_stop + 1)],
                               rtol=1e-12)


def test_residual_stop_rest_and_limits():
    """Fluid at rest: g_0 = u_b, so eps = 1 stops after the first sweep;
    eps = 0 runs every sweep and equals the fixed-count forcing exactly; a
    body at rest (u_b = 0, U = 0) converges at once."""
    rng = np.random.default_rng(3)
    shape = (9, 8, 7)
    p = O.params(shape, 0.7)
    x = rng.uniform([2, 2, 2], [7, 6, 5], size=(20, 3))
    ub = rng.normal(scale=0.01, size=(20, 3))
    s = rng.uniform(0.5, 1.0, 20)
    U0 = np.zeros((3,) + shape[::-1])
    one = O.ibm_ex(p, x, ub, s, U0, n_iter=6, flags=STOP, eps=1.0)
    assert one["n_sweeps"] == 1
    np.testing.assert_array_equal(one["du"], s[:, None] * ub)
    full = O.ibm_ex(p, x, ub, s, U0, n_iter=6, flags=STOP, eps=0.0)
    fixed = O.ibm_ex(p, x, ub, s, U0, n_iter=6)
    assert full["n_sweeps"] == fixed["n_sweeps"] == 6
    # (the oracle's spread adds with atomics: equal up to rounding order)
    np.testing.assert_allclose(full["G"], fixed["G"], rtol=1e-13, atol=1e-18)
    still = O.ibm_ex(p, x, np.zeros_like(ub), s, U0, n_iter=6, flags=STOP, eps=1e-3)
    assert still["n_sweeps"] == 1 and not still["G"].any()


# ---------------------------------------------------------- neighbour lists
def test_neighbours_square_grid():
    """Points of a square grid of spacing 1/2 (exact in binary, so equal
    distances tie exactly): within distance 2 lie the offsets (i, j) with
    i^2 + j^2 < 16; the 16 nearest are the 12 with i^2 + j^2 <= 4 followed
    by the 4 lowest-index ones of the 8 at i^2 + j^2 = 5."""
    n = 9
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rest = np.stack([0.5 * ii.ravel(), 0.5 * jj.ravel(), np.zeros(n * n)], -1)
    nbr = O.neighbours(rest, [0, n * n])
    c = 4 * n + 4                                        # centre point (4, 4)
    got = nbr[c]
    assert (got >= 0).all()
    off = [(int(ii.ravel()[q]) - 4, int(jj.ravel()[q]) - 4) for q in got]
    r2 = [a * a + b * b for a, b in off]
    assert sorted(r2[:12]) == r2[:12] and max(r2[:12]) == 4 and len(set(off[:12])) == 12
    assert all(v == 5 for v in r2[12:])
    ring5 = sorted(q for q in range(n * n)
                   if (ii.ravel()[q] - 4) ** 2 + (jj.ravel()[q] - 4) ** 2 == 5)
    assert list(got[12:]) == ring5[:4]
    # a corner point sees the 14 offsets with i, j >= 0 and i^2 + j^2 < 16
    corner = nbr[0]
    assert (corner >= 0).sum() == 14
    assert (corner[14:] == -1).all()                     # -1 pads after the last one


def test_neighbours_other_bodies_and_far_points():
    """Points of another body never appear, however close; a point with no
    same-body point within distance 2 has an empty list; listed rows match
    the full computation."""
    rng = np.random.default_rng(8)
    a = rng.uniform(-1.5, 1.5, size=(40, 3))
    b = a + 1e-3                                         # body 1, almost on top of body 0
    far = np.array([[50.0, 0.0, 0.0]])
    rest = np.concatenate([a, far, b]).astype(np.float32).astype(np.float64)
    off = [0, 41, 81]
    nbr = O.neighbours(rest, off)
    for k in range(41):
        assert ((nbr[k] < 41) | (nbr[k] == -1)).all() and (nbr[k] != k).all()
    for k in range(41, 81):
        assert ((nbr[k] >= 41) | (nbr[k] == -1)).all()
    assert (nbr[40] == -1).all()
    idx = np.array([3, 40, 55])
    part = O.neighbours(rest, off, idx)
    np.testing.assert_array_equal(part[idx], nbr[idx])
    # the lists are ordered by distance and every member lies within 2
    for k in range(81):
        q = nbr[k][nbr[k] >= 0]
        d = np.sqrt(((rest[q] - rest[k]) ** 2).sum(1))
        assert (d < 2).all() and (np.diff(d) >= 0).all()


# ------------------------------------------------------- features and v_ref
def test_vref_closed_form():
    rest = np.array([[3.0, 4.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 2.0]])
    bodies = np.array([[0, 0, 0, 0, 0, 1, 0.0, -0.01], [0, 0, 0, 0, 0, 1, 0.0, 0.0]])
    v = O.vref(rest, [0, 2, 3], bodies)
    np.testing.assert_allclose(v, [0.05, 1.0], rtol=1e-15)


def test_features_special_cases():
    """Constant deficit: mean = max = the deficit; the component-wise max of
    two neighbours; an empty list gives zeros; everything scales by 1/v."""
    g0 = np.array([[1.0, -2.0, 3.0], [4.0, 5.0, -6.0], [-7.0, 8.0, 9.0], [0.5, 0.5, 0.5]])
    ub = np.arange(12.0).reshape(4, 3)
    nbr = np.full((4, 16), -1, dtype=np.int32)
    nbr[0, :2] = [1, 2]
    nbr[1, :1] = [0]
    v = np.array([2.0, 2.0, 4.0, 1.0])
    f = O.features(g0, ub, nbr, v)
    np.testing.assert_array_equal(f[0, :3], g0[0] / 2)
    np.testing.assert_array_equal(f[0, 3:6], ub[0] / 2)
    np.testing.assert_allclose(f[0, 6:9], (g0[1] + g0[2]) / 2 / 2, rtol=1e-15)
    np.testing.assert_array_equal(f[0, 9:12], np.array([4.0, 8.0, 9.0]) / 2)
    np.testing.assert_array_equal(f[1, 6:9], g0[0] / 2)
    np.testing.assert_array_equal(f[1, 9:12], g0[0] / 2)
    np.testing.assert_array_equal(f[2, 6:], 0.0)
    np.testing.assert_array_equal(f[3, :3], g0[3])


# --------------------------------------------------------------- warm start
def _probe_matrix(p, x):
    nz, ny, nx = p.nz, p.ny, p.nx
    n = nx * ny * nz
    D = np.zeros((len(x), n))
    for c in range(n):
        U = np.zeros((3, n))
        U[0, c] = 1.0
        D[:, c] = O.interpolate(p, x, U.reshape(3, nz, ny, nx))[:, 0]
    return D


def _bias_theta(c):
    th = np.zeros(NP)
    th[-3:] = c
    return th


def test_warm_start_matrix_form():
    """With a network whose output is the constant c (bias only), the warm
    start sets du_1 = s v c and U_1 = U_0 + D^T du_1; the later sweeps follow
    g_n = (I - M) g_{n-1} from g_1 = u_b - D U_1, du = du_1 + s sum_{n>=1} g_n
    and G = D^T du (M = D D^T diag(s), D found by probing)."""
    shape = (6, 5, 7)
    nx, ny, nz = shape
    p = O.params(shape, 0.7)
    rng = np.random.default_rng(21)
    x = rng.uniform(0, 1, size=(10, 3)) * [nx, ny, nz]
    s = rng.uniform(0.3, 1.2, 10)
    ub = rng.normal(scale=0.02, size=(10, 3))
    U0 = rng.normal(scale=0.01, size=(3, nz, ny, nx))
    v = np.full(10, 0.037)
    nbr = np.full((10, 16), -1, dtype=np.int32)
    c = np.array([0.3, -0.2, 0.5])
    N = 4
    r = O.ibm_ex(p, x, ub, s, U0, n_iter=N, flags=WARM, theta=_bias_theta(c), nbr=nbr, v_pt=v)
    D = _probe_matrix(p, x)
    M = D @ D.T @ np.diag(s)
    du1 = (s * v)[:, None] * c[None, :]
    U1 = U0.reshape(3, -1).T + D.T @ du1
    g = [ub - D @ U1]
    for _ in range(N - 2):
        g.append((np.eye(10) - M) @ g[-1])
    du = du1 + s[:, None] * sum(g)
    assert r["n_sweeps"] == N
    np.testing.assert_allclose(r["du"], du, atol=1e-14)
    np.testing.assert_allclose(r["G"].reshape(3, -1), (D.T @ du).T, atol=1e-14)
    np.testing.assert_allclose(r["g"], g[-1], atol=1e-14)


def test_warm_start_zero_network_wastes_one_sweep():
    """A network that predicts 0 leaves U_1 = U_0: N warm-started sweeps give
    the forcing of N - 1 plain sweeps, and sweep n + 1's residual is plain
    sweep n's."""
    rng = np.random.default_rng(5)
    shape = (9, 8, 7)
    p = O.params(shape, 0.7)
    x = rng.uniform([2, 2, 2], [7, 6, 5], size=(30, 3))
    ub = rng.normal(scale=0.01, size=(30, 3))
    s = rng.uniform(0.5, 1.0, 30)
    U0 = rng.normal(scale=0.005, size=(3,) + shape[::-1])
    nbr = np.full((30, 16), -1, dtype=np.int32)
    warm = O.ibm_ex(p, x, ub, s, U0, n_iter=5, flags=WARM, theta=np.zeros(NP), nbr=nbr,
                    v_pt=np.ones(30))
    plain = O.ibm_ex(p, x, ub, s, U0, n_iter=4)
    np.testing.assert_allclose(warm["G"], plain["G"], rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(warm["du"], plain["du"], rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(warm["resid"][1:], plain["resid"], rtol=1e-12)


def test_warm_start_skipped_when_first_sweep_converges():
    """If the first sweep already meets the threshold the prediction is not
    used: the result equals the plain forcing's."""
    rng = np.random.default_rng(9)
    shape = (9, 8, 7)
    p = O.params(shape, 0.7)
    x = rng.uniform([2, 2, 2], [7, 6, 5], size=(12, 3))
    ub = rng.normal(scale=0.01, size=(12, 3))
    s = np.ones(12)
    U0 = np.zeros((3,) + shape[::-1])
    nbr = np.full((12, 16), -1, dtype=np.int32)
    w = O.ibm_ex(p, x, ub, s, U0, n_iter=5, flags=WARM | STOP, eps=1.0,
                 theta=_bias_theta([1.0, 2.0, 3.0]), nbr=nbr, v_pt=np.ones(12))
    pl = O.ibm_ex(p, x, ub, s, U0, n_iter=5, flags=STOP, eps=1.0)
    assert w["n_sweeps"] == pl["n_sweeps"] == 1
    np.testing.assert_allclose(w["G"], pl["G"], rtol=1e-13, atol=1e-18)


def test_step_features_match_function():
    """The features a full step reports are those of its first sweep's
    deficit, with the neighbour lists and reference speeds of the surface."""
    from paper_1904_02108_amd import workload as W
    wl = W.config("c0")
    p = O.params(wl.shape, wl.tau, bc=wl.bc)
    pts = O.Points(wl.rest, wl.area, wl.body_off, wl.bodies, 2, 0)
    f = O.init_equilibrium(p)
    r = O.step(p, f, pts, 3, features=True)
    x, ub = O.kinematics(wl.rest, wl.body_off, wl.bodies, 3)
    # g0 = u_b at rest
    nbr = O.neighbours(wl.rest, wl.body_off)
    vp = O.vref_points(wl.rest, wl.body_off, wl.bodies)
    np.testing.assert_allclose(r["feat"], O.features(ub, ub, nbr, vp), rtol=1e-13, atol=1e-16)
