"""GPU parity of the volume-weighted residual norm (hr_set_residual_norm with
HR_NORM_VOLUME) against the oracle's, on the same seeded workloads.

The norm is sqrt(sum H^2 dV / sum dV) with dV the proper cell volume. It is
compared with the oracle after equal step counts (bar: the same relative
tolerance as the point norm's residual parity, 1e-7, set by the cancellation
inside H), on the resident kernel's grids and on ragged ones, and the relaxing
call's stop test must stop at the check where the oracle's volume norm first
drops below the tolerance.
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_grid

pytestmark = pytest.mark.gpu

RTOL = 1e-7

SPECS = [
    (workloads.GridSpec(0, 32, 16, 4, 8, bscale=1.0), "SinhSymTP 32x16x4 (resident)"),
    (workloads.GridSpec(0, 37, 19, 6, 10, bscale=1.0), "ragged SinhSymTP order 10"),
    (workloads.GridSpec(1, 33, 18, 6, 8, rmax=50.0), "ragged Spherical order 8"),
    (workloads.GridSpec(2, 64, 32, 8, 8), "SinhSpherical 64x32x8 (resident)"),
]


def _pair(spec):
    pz = workloads.equal_mass_small().punctures
    og = oracle_grid(spec)
    og.set_punctures(*pz.as_tuple())
    gg = gpu_grid(spec)
    gg.set_punctures(*pz.as_tuple())
    return og, gg, og.suggest_dt(0.5)


@pytest.mark.parametrize("spec,label", SPECS)
def test_volume_norm_parity(spec, label):
    banner(f"volume norm parity {label}")
    og, gg, dt = _pair(spec)
    gg.set_residual_norm(hr.NORM_VOLUME)
    # the initial state (u = 0): H is the source term alone
    np.testing.assert_allclose(gg.residual_l2(), og.residual_volume(), rtol=1e-13)
    eta = 8.0
    og.relax(eta, 1.0, dt, 300, 0.0, 100)
    res = gg.relax(eta, 1.0, dt, 300, 0.0, check_every=100)
    assert res.status == hr.OK and res.steps_taken == 300
    rv = gg.residual_l2()
    np.testing.assert_allclose(rv, og.residual_volume(), rtol=RTOL)
    # the call's own last check used the volume norm too
    np.testing.assert_allclose(res.history[-1], rv, rtol=1e-14)
    # switching back gives the point norm of the same state
    gg.set_residual_norm(hr.NORM_POINTS)
    np.testing.assert_allclose(gg.residual_l2(), og.residual(), rtol=RTOL)
    assert abs(rv - og.residual()) > 1e-3 * og.residual()


@pytest.mark.parametrize("spec,label", [SPECS[0], SPECS[1]])
def test_volume_norm_stop_test(spec, label):
    banner(f"volume norm stop test {label}")
    og, gg, dt = _pair(spec)
    gg.set_residual_norm(hr.NORM_VOLUME)
    eta, K = 8.0, 100
    # the oracle's volume norm at every check, until well past the tolerance
    hist = []
    for _ in range(40):
        og.relax(eta, 1.0, dt, K, 0.0, K)
        hist.append(og.residual_volume())
    # a tolerance between two checks on the decaying part, far from either and
    # far above the roundoff floor
    tol = float(np.sqrt(hist[3] * hist[4]))
    n_expect = K * (1 + next(k for k, r in enumerate(hist) if r < tol))
    res = gg.relax(eta, 1.0, dt, 40 * K, tol, check_every=K)
    assert res.status == hr.OK
    assert res.steps_taken == n_expect
    # once the norm nears the FP64 floor of H (~1e-10 of the first check's norm
    # here), the two summation orders differ at that level
    np.testing.assert_allclose(res.history, hist[:len(res.history)], rtol=RTOL,
                               atol=1e-10 * hist[0])


@pytest.mark.parametrize("spec,label", [SPECS[0], SPECS[2]])
def test_volume_norm_integration_radius(spec, label):
    banner(f"volume norm with integration radius {label}")
    og, gg, dt = _pair(spec)
    X, Y, Z = og.cart()
    ri = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)[og.NG, og.NG:-og.NG, og.NG:-og.NG]
    # about half of the cells inside; the radius sits halfway between two cell
    # centre distances so that no cell is a rounding-dependent tie
    # (distances equal up to rounding, e.g. one Spherical shell, are merged)
    scale = float(ri.max())
    rs = np.unique(np.round(ri / scale, 9)) * scale
    k = len(rs) // 2
    R = 0.5 * float(rs[k] + rs[k + 1])
    gg.set_residual_norm(hr.NORM_VOLUME, R)
    np.testing.assert_allclose(gg.residual_l2(), og.residual_volume(R), rtol=1e-13)
    og.relax(8.0, 1.0, dt, 300, 0.0, 100)
    res = gg.relax(8.0, 1.0, dt, 300, 0.0, check_every=100)
    assert res.status == hr.OK
    rv = gg.residual_l2()
    banner(f"radius {R:.6g}: gpu {rv:.12e} oracle {og.residual_volume(R):.12e}")
    np.testing.assert_allclose(rv, og.residual_volume(R), rtol=RTOL)
    np.testing.assert_allclose(res.history[-1], rv, rtol=1e-14)
    # another radius on the same state, then the whole grid again
    R2 = 0.5 * float(rs[-2] + rs[-1])  # all but the outermost cells
    gg.set_residual_norm(hr.NORM_VOLUME, R2)
    banner(f"radius {R2:.6g}: gpu {gg.residual_l2():.12e} oracle {og.residual_volume(R2):.12e}")
    np.testing.assert_allclose(gg.residual_l2(), og.residual_volume(R2), rtol=RTOL)
    gg.set_residual_norm(hr.NORM_VOLUME)
    np.testing.assert_allclose(gg.residual_l2(), og.residual_volume(), rtol=RTOL)


def test_volume_norm_errors():
    banner("volume norm errors")
    spec = SPECS[0][0]
    _, gg, _ = _pair(spec)
    with pytest.raises(hr.HRError):
        gg.set_residual_norm(2)
    with pytest.raises(hr.HRError):
        gg.set_residual_norm(hr.NORM_POINTS, 1.0)     # a radius needs the volume norm
    with pytest.raises(hr.HRError):
        gg.set_residual_norm(hr.NORM_VOLUME, 1e-9)    # no cell centre inside
    with pytest.raises(hr.HRError):
        gg.set_residual_norm(hr.NORM_VOLUME, float("nan"))
    gg.set_residual_norm(hr.NORM_VOLUME)
    b = hr.Batch([gg])
    try:
        with pytest.raises(hr.HRError) as e:
            b.relax([8.0], 1.0, n_steps=100, tol=0.0, check_every=100)
        assert e.value.status == hr.EINVAL
        gg.set_residual_norm(hr.NORM_POINTS)
        res = b.relax([8.0], 1.0, n_steps=100, tol=0.0, check_every=100)
        assert res[0].steps_taken == 100
    finally:
        b.close()
