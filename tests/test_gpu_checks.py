"""Failure detection and checkpoint/resume on the GPU, through the C ABI.

* The non-finite check (lbm_set_check): a NaN population written from the
  host is reported as LBM_ERR_NONFINITE by the next checked step; a finite
  but unrepresentable deficit (a velocity far beyond any lattice flow)
  raises the forcing's spread guard; a finite flow passes the check.  The
  conditions are forced from the host; every kernel runs to its normal end.
* Checkpoint/resume: populations read back in FP64, written again and read
  back reproduce the first read bit for bit for every storage format, and a
  run resumed from such a checkpoint agrees with the uninterrupted one to
  rounding (offsets below half an FP64 ulp of t_i do not survive the FP64
  export)."""
import numpy as np
import pytest

import oracle as O
from gpu_common import make_sim, to_np
from paper_1904_02108_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1904_02108_amd import lbmibm
    return lbmibm


def _weights():
    return O.d3q19()[1]


def test_nan_population_reported(L):
    shape = (16, 12, 10)
    sim = make_sim(L, shape, 0.7)
    f = W.random_populations(shape, 3, amp=0.02, weights=_weights())
    f[5, 4, 6, 7] = np.nan
    sim.write(pops=f)
    sim.set_check(1)
    with pytest.raises(L.LbmError) as ei:
        sim.step(1)
    assert ei.value.status == L.LBM_ERR_NONFINITE
    assert "sums not finite" in str(ei.value)
    # the words stay raised until the check is set again; with the check off
    # the (non-finite) run goes on without an error
    with pytest.raises(L.LbmError):
        sim.step(1)
    sim.set_check(0)
    sim.step(2)
    assert int(to_np(sim.read("step")["step"])[0]) == 4
    sim.close()


def test_finite_flow_passes_check(L):
    wl = W.config("c0")
    sim = make_sim(L, wl.shape, wl.tau, bc=wl.bc, forcing=wl.forcing, max_points=wl.n_points)
    sim.set_points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
    sim.set_check(1)
    sim.step(6)
    sim.force_iterate()
    sim.set_check(3)
    sim.step(6)
    sums = to_np(sim.read("sums")["sums"])
    assert np.isfinite(sums).all()
    sim.close()


def test_spread_guard_reports_out_of_range_deficit(L):
    """Populations with a velocity of 2e4 (finite, far beyond any lattice
    flow) on the support of the surface: the deficit the first sweep spreads
    exceeds the fixed-point range, and the forcing reports it."""
    wl = W.tiny_propeller_case(shape=(24, 20, 28))
    sim = make_sim(L, wl.shape, wl.tau, bc=wl.bc, forcing=wl.forcing, max_points=wl.n_points)
    sim.set_points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
    w = _weights()
    nx, ny, nz = wl.shape
    f = np.broadcast_to(w.reshape(19, 1, 1, 1), (19, nz, ny, nx)).copy()
    x, _ = O.kinematics(wl.rest, wl.body_off, wl.bodies, 0)
    lo = np.floor(x.min(axis=0)).astype(int) - 2
    hi = np.floor(x.max(axis=0)).astype(int) + 3
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    # +x and -x populations moved apart: rho stays 1, rho U_x = 2e4
    f[(1,) + sl] += 1e4
    f[(2,) + sl] -= 1e4
    sim.write(pops=f)
    sim.set_check(1)
    with pytest.raises(L.LbmError) as ei:
        sim.force_iterate()
    assert ei.value.status == L.LBM_ERR_NONFINITE
    msg = str(ei.value)
    assert "spread value" in msg and "sums not finite" not in msg
    sim.close()


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["f32", "f16", "bf16"])
@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 1)], ids=["periodic", "walls"])
def test_checkpoint_round_trip_bit_exact(L, storage, bc):
    """Read POPS -> write POPS -> read POPS is bit-exact.  The export holds
    full populations t_i + (f_i - t_i) in FP64, so a stored offset smaller
    than half an FP64 ulp of t_i (about 3e-17; FP32 and BF16 offsets near zero
    can be) does not survive the round trip: the resumed run then agrees with
    the uninterrupted one to rounding (1e-12 of each field's peak), not bit
    for bit."""
    wl = W.config("c0")
    shape = (32, 32, 32)
    sim = make_sim(L, shape, wl.tau, bc=bc, storage=storage, forcing=wl.forcing,
                   max_points=wl.n_points)
    sim.set_points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
    sim.step(7)
    p1 = to_np(sim.read("pops", pops_f64=True)["pops"])
    sim.write(pops=p1)
    p2 = to_np(sim.read("pops", pops_f64=True)["pops"])
    np.testing.assert_array_equal(p1, p2)
    # resume: a second run stepped straight through ends in the same state
    sim.step(5)
    a = sim.read("vel", "force", "pops", "pt_du")
    sim.close()
    ref = make_sim(L, shape, wl.tau, bc=bc, storage=storage, forcing=wl.forcing,
                   max_points=wl.n_points)
    ref.set_points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
    ref.step(12)
    b = ref.read("vel", "force", "pops", "pt_du")
    ref.close()
    for k in ("vel", "force", "pops", "pt_du"):
        x, y = to_np(a[k]).astype(np.float64), to_np(b[k]).astype(np.float64)
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max(), k
