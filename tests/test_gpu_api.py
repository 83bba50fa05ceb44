"""GPU tests of the C ABI's state handling, control flow and error paths."""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu


def _config0():
    w = workloads.equal_mass_small()
    g = gpu_grid(w.grid)
    g.set_punctures(*w.punctures.as_tuple())
    return w, g


def test_resume_is_bitwise():
    banner("checkpoint/resume bitwise")
    w, a = _config0()
    a.relax(w.eta, 1.0, 0.0, 200, 0.0, check_every=100)
    w, b = _config0()
    b.relax(w.eta, 1.0, 0.0, 100, 0.0, check_every=100)
    u = b.get_u(extended=True)
    v = b.get_v(extended=True)
    w, c = _config0()
    c.set_u(u)
    c.set_v(v)
    c.relax(w.eta, 1.0, 0.0, 100, 0.0, check_every=100)
    assert np.array_equal(a.get_u(extended=True), c.get_u(extended=True))
    assert np.array_equal(a.get_v(extended=True), c.get_v(extended=True))


def test_interior_layout_and_outer_continuation():
    banner("interior get/set layout")
    w, g = _config0()
    N0, N1, N2 = w.grid.shape
    ng = w.grid.fd_order // 2
    rng = np.random.default_rng(3)
    ui = rng.uniform(0.1, 0.2, size=(N2, N1, N0))
    g.set_u(ui)
    back = g.get_u()
    assert np.array_equal(back, ui)
    ext = g.get_u(extended=True)
    assert np.array_equal(ext[:, :, :N0], ui)
    # outer points follow f * r = const along each x0 row
    og = oracle_grid(w.grid)
    X, Y, Z = og.cart()
    r = oracle_extended(og, np.sqrt(X ** 2 + Y ** 2 + Z ** 2))
    prod = ext[:, :, N0 - 1:] * r[:, :, N0 - 1:]
    np.testing.assert_allclose(prod, prod[:, :, :1].repeat(ng + 1, axis=2), rtol=1e-13)


def test_warm_start_matches_oracle():
    banner("warm start parity")
    w = workloads.equal_mass_small()
    og = oracle_grid(w.grid)
    og.set_punctures(*w.punctures.as_tuple())
    og.relax(w.eta, 1.0, og.suggest_dt(0.5), 300, 0.0, 100)
    u0, v0 = og.state()
    g = gpu_grid(w.grid)
    g.set_punctures(*w.punctures.as_tuple())
    g.set_u(oracle_extended(og, u0))
    g.set_v(oracle_extended(og, v0))
    og.relax(w.eta, 1.0, og.suggest_dt(0.5), 300, 0.0, 100)
    g.relax(w.eta, 1.0, og.suggest_dt(0.5), 300, 0.0, check_every=100)
    ou, _ = og.state()
    assert rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou)) <= 1e-12


def test_tolerance_stop_and_history():
    banner("tolerance stop")
    w, g = _config0()
    og = oracle_grid(w.grid)
    og.set_punctures(*w.punctures.as_tuple())
    st, n, hist = og.relax(8.0, 1.0, og.suggest_dt(0.5), 20000, 1e-11, 100)
    assert st == 0
    res = g.relax(8.0, 1.0, 0.0, 20000, 1e-11, check_every=100)
    assert res.status == hr.OK
    assert res.steps_taken == n
    assert res.residual < 1e-11
    np.testing.assert_allclose(res.history, hist, rtol=1e-6, atol=1e-15)


def test_not_converged_and_nonfinite_statuses():
    banner("ENOTCONV / ENONFINITE")
    w, g = _config0()
    res = g.relax(1.0, 1.0, 0.0, 300, 1e-30, check_every=100)
    assert res.status == hr.ENOTCONV and res.steps_taken == 300
    dt = g.suggest_dt(0.5)
    w, g = _config0()
    res = g.relax(1.0, 1.0, 50 * dt, 2000, 0.0, check_every=50, raise_on_error=False)
    assert res.status == hr.ENONFINITE
    assert not np.isfinite(res.history[-1])


def test_state_errors():
    banner("ESTATE / EINVAL")
    w = workloads.equal_mass_small()
    g = gpu_grid(w.grid)
    with pytest.raises(hr.HRError) as e:
        g.relax(1.0, 1.0, 0.0, 10, 0.0)
    assert e.value.status == hr.ESTATE
    with pytest.raises(hr.HRError) as e:
        g.set_punctures([0.5, -0.5], [[0, 0, 1], [0, 0, -1]], np.zeros((2, 3)), np.zeros((2, 3)))
    assert e.value.status == hr.EINVAL
    with pytest.raises(hr.HRError) as e:
        g.set_u(np.zeros(7))
    assert e.value.status == hr.EINVAL
    g.set_punctures(*w.punctures.as_tuple())
    with pytest.raises(hr.HRError) as e:
        g.relax(-1.0, 1.0, 0.0, 10, 0.0)
    assert e.value.status == hr.EINVAL


def test_launch_timing_counts_the_resident_launches():
    """hr_set_launch_timing times each resident launch hr_relax issues: ten
    100-step intervals are ten launches of 400 stages, and their summed
    durations fit inside the call's wall time."""
    import time

    w = workloads.paper_scale()
    g = gpu_grid(w.grid)
    g.set_punctures(*w.punctures.as_tuple())
    assert g.resolved_kernel(hr.FP64)["variant"] == 3
    g.relax(w.eta, 1.0, 0.0, 100, 0.0, check_every=100)      # warm-up
    g.set_launch_timing(True)
    t0 = time.perf_counter()
    r = g.relax(w.eta, 1.0, 0.0, 1000, 0.0, check_every=100)
    wall = time.perf_counter() - t0
    t = g.launch_timing()
    banner(f"launch timing {t}, wall {wall * 1e3:.2f} ms")
    assert r.status == hr.OK
    assert t["launches"] == 10 and t["stages"] == 4000
    assert 0.0 < t["total_us"] * 1e-6 <= wall
    g.set_launch_timing(False)
    g.relax(w.eta, 1.0, 0.0, 100, 0.0, check_every=100)
    assert g.launch_timing()["launches"] == 0
