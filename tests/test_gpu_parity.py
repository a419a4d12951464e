"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerance (relative L-infinity, max|gpu - oracle| / max|oracle| per field):
1e-5 for one step from an identical state, 1e-4 after 100 steps, for FP32
population storage.  Inputs are seeded; the oracle sees exactly the values
the GPU was given (FP32 populations are written as FP64 and rounded once on
the GPU; point data are FP32 for both)."""
import numpy as np
import pytest

import oracle as O
from gpu_common import make_sim, oracle_params, rel_linf, sim_for_workload, to_np, wrap_diff
from paper_1904_02108_amd import workload as W

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5
TOL_100 = 1e-4


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1904_02108_amd import lbmibm
    return lbmibm


@pytest.fixture(scope="module")
def lat():
    return O.d3q19()


def _rand_pops(shape, seed, lat, amp=0.05):
    _, w, _ = lat
    return W.random_populations(shape, seed, amp=amp, weights=w)


def _offsets(f, lat):
    _, w, _ = lat
    return f - w.reshape(19, 1, 1, 1)


# ---------------------------------------------------------------- lattice only
@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_initial_state(L, lat, bc):
    shape = (9, 8, 7)
    u0 = (0.02, -0.01, 0.03)
    wu = np.zeros((3, 2, 3))
    wu[1, 1] = [0.01, 0.0, -0.02]
    sim = make_sim(L, shape, 0.7, bc=bc, u0=u0, rho0=1.02, wall_u=wu, rho_wall=1.0)
    f = to_np(sim.read("pops", pops_f64=True)["pops"])
    p = oracle_params(shape, 0.7, bc=bc)
    ref = O.init_equilibrium(p, 1.02, u0)
    assert np.abs(f - ref).max() < 1e-7


CASES = [
    dict(shape=(13, 10, 9), bc=(0, 0, 0), forcing=0, tau=0.6),
    dict(shape=(16, 16, 16), bc=(0, 0, 0), forcing=1, tau=0.55),
    dict(shape=(12, 9, 11), bc=(0, 1, 1), forcing=0, tau=0.8, moving=True),
    dict(shape=(7, 12, 10), bc=(1, 1, 1), forcing=1, tau=0.9, moving=True, g_ext=(1e-5, -2e-5, 3e-5)),
    dict(shape=(5, 3, 7), bc=(0, 0, 1), forcing=0, tau=0.7),
    # even x extents with walls on x, rows that end inside a wavefront, and
    # nx = 2, where both x neighbours of a cell wrap or meet a wall
    dict(shape=(8, 12, 10), bc=(1, 1, 1), forcing=0, tau=0.9, moving=True),
    dict(shape=(10, 7, 6), bc=(1, 0, 1), forcing=1, tau=0.7),
    dict(shape=(130, 3, 2), bc=(0, 0, 0), forcing=0, tau=0.65),
    dict(shape=(2, 5, 4), bc=(0, 0, 0), forcing=1, tau=0.6),
    dict(shape=(2, 6, 3), bc=(1, 1, 0), forcing=0, tau=0.75),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c["shape"])) + "-bc" +
                         "".join(map(str, c["bc"])) + ("-shift" if c["forcing"] else "-guo"))
def test_stream_collide_one_step(L, lat, case):
    shape, bc, forcing, tau = case["shape"], case["bc"], case["forcing"], case["tau"]
    wu = None
    if case.get("moving"):
        wu = np.zeros((3, 2, 3))
        wu[1, 1] = [0.02, 0.0, 0.01]
        wu[2, 0] = [-0.01, 0.015, 0.0]
    g_ext = case.get("g_ext", (0.0, 0.0, 0.0))
    sim = make_sim(L, shape, tau, bc=bc, forcing=forcing, wall_u=wu, rho_wall=1.0, g_ext=g_ext)
    f0 = _rand_pops(shape, 11, lat)
    G = W.random_field(shape, 12, amp=2e-3)
    sim.write(pops=f0, force=G)
    sim.step(1)
    out = sim.read("pops", "rho", "vel", "sums", pops_f64=True)
    p = oracle_params(shape, tau, bc=bc, forcing=forcing, wall_u=wu, g_ext=g_ext)
    ref = O.collide_stream(p, f0, G)
    rho_r, U_r = O.moments(p, ref)
    assert rel_linf(_offsets(to_np(out["pops"]), lat), _offsets(ref, lat)) < TOL_STEP
    assert rel_linf(to_np(out["rho"]) - 1.0, rho_r - 1.0) < 1e-4   # FP32 rho = 1 + drho
    assert rel_linf(to_np(out["vel"]), U_r) < TOL_STEP
    s_ref = O.sums(p, f0)   # sums of the state the step started from
    s = to_np(out["sums"])
    assert abs(s[0] - s_ref[0]) < 1e-9 * s_ref[0]
    assert np.abs(s[1:] - s_ref[1:]).max() < 1e-6


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_rest_state_exact(L, lat, storage):
    shape = (16, 8, 12)
    sim = make_sim(L, shape, 0.6, bc=(0, 1, 0), storage=storage)
    sim.step(10)
    f = to_np(sim.read("pops", pops_f64=True)["pops"])
    _, w, _ = lat
    np.testing.assert_array_equal(f, np.broadcast_to(w.reshape(19, 1, 1, 1), f.shape))


def test_conservation_gpu(L, lat):
    """Mass conserved and momentum changed by sum rho G, from the FP64 sums."""
    shape = (16, 12, 8)
    sim = make_sim(L, shape, 0.7, forcing=0)
    f0 = _rand_pops(shape, 21, lat, amp=0.02)
    G = W.random_field(shape, 22, amp=1e-3)
    sim.write(pops=f0, force=G)
    rho = to_np(sim.read("rho")["rho"]).astype(np.float64)   # density of state 0
    sim.step(1)
    s0 = to_np(sim.read("sums")["sums"])   # sums of state 0
    sim.step(1)
    s1 = to_np(sim.read("sums")["sums"])   # sums of state 1
    assert abs(s1[0] - s0[0]) < 1e-10 * s0[0] + 1e-4
    np.testing.assert_allclose(s1[1:] - s0[1:], (rho[None] * G).sum(axis=(1, 2, 3)), rtol=2e-4, atol=1e-6)


# --------------------------------------------------------------- forcing
def _tiny(bc=(0, 0, 0), shape=(24, 20, 28), forcing=0):
    return W.tiny_propeller_case(shape=shape, bc=bc, forcing=forcing)


FORCE_CASES = {
    "tiny-periodic": lambda: _tiny(),
    "tiny-walls": lambda: _tiny(bc=(0, 1, 1), shape=(24, 22, 26)),
    "tiny-shift": lambda: _tiny(forcing=1, shape=(21, 19, 17)),
    "c0": lambda: W.config("c0"),
}


def _check_forcing(sim, p, pts, wl, step, U0, tol=TOL_STEP):
    x_r, ub_r = O.kinematics(wl.rest, wl.body_off, wl.bodies, step)
    G_r, du_r, g_r, res_r = O.ibm(p, x_r, ub_r, wl.area, U0, wl.n_iter, pts.flags)
    st = sim.force_iterate(stats=True)
    out = sim.read("force", "pt_x", "pt_ub", "pt_g", "pt_du")
    assert np.abs(wrap_diff(to_np(out["pt_x"]), x_r, wl.shape, wl.bc)).max() < 1e-5
    assert rel_linf(to_np(out["pt_ub"]), ub_r) < 1e-6
    assert rel_linf(to_np(out["force"]), G_r) < tol
    assert rel_linf(to_np(out["pt_du"]), du_r) < tol
    assert rel_linf(to_np(out["pt_g"]), g_r) < 10 * tol    # last deficit is a small difference
    np.testing.assert_allclose(st["resid"], res_r, rtol=1e-4)
    assert abs(st["sum_s"] - wl.area.astype(np.float64).sum()) < 1e-9 * st["sum_s"]
    return G_r


@pytest.mark.parametrize("name", list(FORCE_CASES))
@pytest.mark.parametrize("flags", [0, 1])
def test_forcing_from_rest(L, name, flags):
    wl = FORCE_CASES[name]()
    sim, p, pts = sim_for_workload(L, wl, flags=flags)
    U0 = np.zeros((3,) + tuple(reversed(wl.shape)))
    _check_forcing(sim, p, pts, wl, 0, U0)


@pytest.mark.parametrize("name", ["tiny-periodic", "tiny-walls"])
def test_forcing_on_random_flow(L, lat, name):
    """Forcing with a nonzero velocity field and a step index > 0."""
    wl = FORCE_CASES[name]()
    sim, p, pts = sim_for_workload(L, wl)
    f0 = _rand_pops(wl.shape, 31, lat, amp=0.03)
    sim.write(pops=f0, step=7)
    _, U0 = O.moments(p, f0)
    _check_forcing(sim, p, pts, wl, 7, U0)


U_STRATEGIES = {"tile-mask": 0, "box": 64, "kernel": 128}


@pytest.mark.parametrize("name", ["tiny-periodic", "tiny-walls"])
@pytest.mark.parametrize("strategy", list(U_STRATEGIES))
def test_u_prepass_strategy_on_random_flow(L, lat, name, strategy):
    """Each U pre-pass strategy (§5: box, kernel, and the default tile mask)
    against the oracle on a random flow at step 7."""
    wl = FORCE_CASES[name]()
    sim, p, _ = sim_for_workload(L, wl, flags=U_STRATEGIES[strategy])
    pts = O.Points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter, 0)
    f0 = _rand_pops(wl.shape, 33, lat, amp=0.03)
    sim.write(pops=f0, step=7)
    _, U0 = O.moments(p, f0)
    _check_forcing(sim, p, pts, wl, 7, U0)


@pytest.mark.parametrize("name,steps", [("c0", 4), ("paper18", 2)])
def test_u_prepass_strategies_identical(L, name, steps):
    """The three U pre-pass strategies compute the same U wherever it is
    read, with the same arithmetic: force, corrections and the flow after a
    few steps are bit-identical."""
    wl = W.config(name)
    out = {}
    for strategy, flags in U_STRATEGIES.items():
        sim, _, _ = sim_for_workload(L, wl, flags=flags)
        sim.step(steps)
        out[strategy] = {k: to_np(v) for k, v in sim.read("force", "pt_du", "vel").items()}
        sim.close()
    for strategy in ("box", "kernel"):
        for k in ("force", "pt_du", "vel"):
            assert np.array_equal(out[strategy][k], out["tile-mask"][k]), (strategy, k)


def test_special_positions(L, lat):
    """Non-rotating points at integer and half-integer coordinates and on the
    periodic seams, on a box smaller than one tile along y."""
    shape = (11, 5, 9)
    x = W.random_points(shape, 40, 41)
    c = np.array([5.0, 2.0, 4.0])
    rest = (x - c).astype(np.float32)
    area = np.linspace(0.3, 1.2, 40).astype(np.float32)
    bodies = np.array([[c[0], c[1], c[2], 0.0, 0.0, 1.0, 0.0, 0.0]])
    wl = W.Workload("special", shape, 0.7, (0, 0, 0), 0, rest, area, np.array([0, 40]), bodies, 5, 1)
    sim, p, pts = sim_for_workload(L, wl)
    f0 = _rand_pops(shape, 42, lat, amp=0.03)
    sim.write(pops=f0)
    _, U0 = O.moments(p, f0)
    _check_forcing(sim, p, pts, wl, 0, U0)


@pytest.mark.parametrize("shape", [(9, 3, 10), (10, 2, 11), (12, 1, 9), (17, 9, 20)])
def test_short_periodic_axes(L, lat, shape):
    """Axes shorter than a support or than a tile, and short last tiles: the
    supports wrap onto the same cells several times; both sides add every
    wrapped tap."""
    x = W.random_points(shape, 30, 81, special=False)
    c = np.array(shape, dtype=np.float64) / 2
    rest = (x - c).astype(np.float32)
    area = np.linspace(0.2, 1.0, 30).astype(np.float32)
    bodies = np.array([[c[0], c[1], c[2], 0.0, 0.0, 1.0, 0.0, 0.0]])
    wl = W.Workload("short", shape, 0.7, (0, 0, 0), 0, rest, area, np.array([0, 30]), bodies, 5, 1)
    sim, p, pts = sim_for_workload(L, wl)
    f0 = _rand_pops(shape, 82, lat, amp=0.03)
    sim.write(pops=f0)
    _, U0 = O.moments(p, f0)
    _check_forcing(sim, p, pts, wl, 0, U0)


def test_multi_body_with_empty_body(L, lat):
    a = W.tiny_propeller_case(shape=(30, 26, 24))
    b = W.tiny_propeller_case(shape=(30, 26, 24), axis=(1, 0.2, 0), omega=-0.03, theta0=1.0,
                              centre=(8.3, 20.1, 6.6))
    n1, n2 = a.n_points, b.n_points
    rest = np.concatenate([a.rest, b.rest])
    area = np.concatenate([a.area, b.area])
    off = np.array([0, n1, n1, n1 + n2])
    bodies = np.concatenate([a.bodies, a.bodies, b.bodies])
    wl = W.Workload("multi", (30, 26, 24), 0.7, (0, 0, 0), 0, rest, area, off, bodies, 4, 1)
    sim, p, pts = sim_for_workload(L, wl)
    f0 = _rand_pops(wl.shape, 51, lat, amp=0.03)
    sim.write(pops=f0, step=3)
    _, U0 = O.moments(p, f0)
    _check_forcing(sim, p, pts, wl, 3, U0)


# ------------------------------------------------------------ whole steps
@pytest.mark.parametrize("name", ["tiny-periodic", "tiny-walls", "tiny-shift"])
def test_full_step_from_oracle_state(L, lat, name):
    wl = FORCE_CASES[name]()
    sim, p, pts = sim_for_workload(L, wl)
    f0 = _rand_pops(wl.shape, 61, lat, amp=0.03)
    sim.write(pops=f0, step=5)
    sim.step(1)
    out = sim.read("pops", "vel", "force", "pt_du", pops_f64=True)
    f = f0.copy()
    r = O.step(p, f, pts, 5)
    _, U_r = O.moments(p, f)
    assert rel_linf(_offsets(to_np(out["pops"]), lat), _offsets(f, lat)) < TOL_STEP
    assert rel_linf(to_np(out["vel"]), U_r) < TOL_STEP
    assert rel_linf(to_np(out["force"]), r["G"]) < TOL_STEP
    assert rel_linf(to_np(out["pt_du"]), r["du"]) < TOL_STEP


def _run_compare(L, wl, n_steps, checkpoints, tol_first=TOL_STEP, tol_last=TOL_100, storage=0):
    sim, p, pts = sim_for_workload(L, wl, storage=storage)
    f = O.init_equilibrium(p)
    done = 0
    errs = {}
    for cp in checkpoints:
        sim.step(cp - done)
        O.run(p, f, pts, done, cp - done - 1)
        r = O.step(p, f, pts, cp - 1)
        done = cp
        out = sim.read("rho", "vel", "force", "pt_du")
        rho_r, U_r = O.moments(p, f)
        errs[cp] = dict(rho=rel_linf(to_np(out["rho"]) - 1, rho_r - 1),
                        vel=rel_linf(to_np(out["vel"]), U_r),
                        force=rel_linf(to_np(out["force"]), r["G"]),
                        du=rel_linf(to_np(out["pt_du"]), r["du"]))
        print(wl.name, cp, errs[cp], flush=True)
    first, last = checkpoints[0], checkpoints[-1]
    for k in ("vel", "force", "du"):
        assert errs[first][k] < tol_first, (first, k, errs[first])
        assert errs[last][k] < tol_last, (last, k, errs[last])
    assert errs[last]["rho"] < 10 * tol_last
    return errs


def test_c0_run(L):
    """C0: 32^3 periodic, one propeller, 5 sweeps: 1 step within 1e-5,
    the full 50-step run and 100 steps within 1e-4."""
    _run_compare(L, W.config("c0"), 100, [1, 50, 100])


def test_c1_first_100_steps(L):
    """C1: 128^3 with walls on y and z, one large propeller (h 0.7)."""
    _run_compare(L, W.config("c1"), 100, [1, 100])


def test_c2_dense_first_steps(L):
    """C2 at full size (256^3, 64 propellers, 1.6M points): two steps from
    rest, every cell and point compared."""
    _run_compare(L, W.config("c2_dense"), 2, [1, 2], tol_last=TOL_STEP)


@pytest.mark.parametrize("n_props", [1, 18])
def test_paper_family_first_steps(L, n_props):
    """The §6 test-case family at full size (160 x 160 x 320, 3930 points per
    propeller): three steps from rest, every cell and point compared."""
    _run_compare(L, W.config("paper%d" % n_props), 3, [1, 3], tol_last=TOL_STEP)


# ---------------------------------------------------------- error paths
def test_error_paths(L):
    shape = (16, 16, 16)
    sim = make_sim(L, shape, 0.6, bc=(0, 1, 0), max_points=10)
    with pytest.raises(L.LbmError) as ei:
        sim.read("sums")
    assert ei.value.status == L.LBM_ERR_STATE
    with pytest.raises(L.LbmError) as ei:
        sim.force_iterate()
    assert ei.value.status == L.LBM_ERR_STATE
    rest = np.array([[0.0, 6.5, 0.0]], dtype=np.float32)
    bodies = np.array([[8.0, 8.0, 8.0, 0, 0, 1, 0.0, 0.01]])
    with pytest.raises(L.LbmError) as ei:       # |r| = 6.5 reaches y = 1.5 .. 14.5 >= n - 2
        sim.set_points(rest, [1.0], [0, 1], bodies)
    assert ei.value.status == L.LBM_ERR_DOMAIN
    with pytest.raises(L.LbmError) as ei:
        sim.set_points(np.zeros((11, 3), np.float32), np.ones(11), [0, 11], bodies)
    assert ei.value.status == L.LBM_ERR_ARG
    with pytest.raises(L.LbmError) as ei:
        sim.set_points(np.zeros((2, 3), np.float32), np.ones(2), [0, 3], bodies)
    assert ei.value.status == L.LBM_ERR_ARG
    with pytest.raises(L.LbmError) as ei:      # two U pre-pass strategies at once
        sim.set_points(np.zeros((2, 3), np.float32), np.ones(2), [0, 2], bodies, 5,
                       L.IBM_U_BOX | L.IBM_U_KERNEL)
    assert ei.value.status == L.LBM_ERR_ARG
    sim.set_points(np.zeros((2, 3), np.float32), np.ones(2), [0, 2], bodies)
    with pytest.raises(L.LbmError) as ei:
        sim.write(force=np.zeros((3, 16, 16, 16), np.float32))
    assert ei.value.status == L.LBM_ERR_STATE
    with pytest.raises(L.LbmError) as ei:
        L.lbm_step(sim.ctx, -1)
    assert ei.value.status == L.LBM_ERR_ARG
    L.lbm_step(sim.ctx, 0)
    sim.step(2)
    st = sim.read("step")["step"]
    assert int(st.item()) == 2
    sim.set_points(np.zeros((0, 3), np.float32), np.zeros(0), [0], bodies[:0])
    sim.step(1)


def test_timing_api(L):
    wl = _tiny()
    sim, _, _ = sim_for_workload(L, wl)
    L.lbm_set_timing(sim.ctx, 1)
    sim.step(5)
    t = L.lbm_get_timing(sim.ctx)
    assert t["n_forcing"] == 5 and t["n_fluid"] == 5
    assert t["ms_forcing"] > 0 and t["ms_fluid"] > 0
