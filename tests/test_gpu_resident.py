"""Resident RK4 kernel (kernel variant 3): whole RK4 steps in one kernel
launch, the state of every 8 x 8 (or 8 x 4) (x0, x1) patch held on chip and
the stage input exchanged between patches through global memory.

It evaluates the stage kernels' arithmetic in the same order, so its
trajectories must agree with the plane-tile kernels to a few roundoff units
and with the oracle to the parity tolerance. The cases cover the paper-scale
grid (256 patches, one per compute unit), 8th and 10th order, Spherical
coordinates (the xx0 reflection pairs patches across the theta range), a
single patch, N2 = 2 (phi taps wrapping several times) and N2 = 14 (idle
plane groups)."""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

CASES = [
    (workloads.GridSpec(0, 128, 128, 16, 10, bscale=5.0), True),
    (workloads.GridSpec(0, 64, 64, 8, 8, bscale=3.0), True),
    (workloads.GridSpec(1, 64, 32, 8, 10, rmax=60.0), True),
    (workloads.GridSpec(0, 16, 8, 2, 10, amax=100.0, sinhwaa=0.2, bscale=1.0), True),
    (workloads.GridSpec(0, 8, 8, 6, 10, amax=100.0, sinhwaa=0.2, bscale=1.0), False),
    (workloads.GridSpec(0, 24, 40, 14, 8, bscale=2.0), False),
    # N1 = 12: only 8 x 4 patches fit
    (workloads.GridSpec(0, 32, 12, 4, 8, amax=100.0, sinhwaa=0.2, bscale=1.0), True),
]


def _punctures(spec):
    D = 2 * spec.bscale if spec.coords == 0 else 10.0
    return workloads.quasi_circular(1.7, D, [0.1, 0.2, 0.3], [0.0, -0.2, 0.1])


def _run(spec, variant, n_steps, dt, eta=6.0, tol=0.0, chunk=0):
    g = gpu_grid(spec)
    g.set_kernel_config(variant=variant, chunk=chunk)
    g.set_punctures(*_punctures(spec).as_tuple())
    r = g.relax(eta, 1.0, dt, n_steps, tol, check_every=100)
    return g, r


def _rows_available(spec):
    """Patch rows (8, 4) the resident kernel accepts for this grid."""
    g = gpu_grid(spec)
    rows = []
    for r in (8, 4):
        try:
            g.set_kernel_config(variant=3, chunk=r)
            rows.append(r)
        except hr.HRError:
            pass
    return rows


@pytest.mark.parametrize("spec,with_oracle", CASES)
def test_resident_matches_plane_kernels_and_oracle(spec, with_oracle):
    banner(f"resident {spec.name()}")
    og = oracle_grid(spec)
    dt = og.suggest_dt(0.5)
    gp, rp = _run(spec, 1, 250, dt)
    ou = None
    if with_oracle:
        og.set_punctures(*_punctures(spec).as_tuple())
        og.relax(6.0, 1.0, dt, 250, 0.0, 100)
        ou, _ = og.state()
    rows = _rows_available(spec)
    assert rows, "no resident partition"
    for r in rows:
        # 250 steps: two checked intervals and an unchecked tail of 50
        gr, rr = _run(spec, 3, 250, dt, chunk=r)
        assert gr.resolved_kernel(hr.FP64)["chunk"] == r
        assert rr.status == hr.OK and rr.steps_taken == 250
        du = rel_maxdiff(gr.get_u(extended=True), gp.get_u(extended=True))
        dv = rel_maxdiff(gr.get_v(extended=True), gp.get_v(extended=True))
        banner(f"resident (8 x {r} patches) vs plane: u {du:.2e}, v {dv:.2e}")
        # same arithmetic, contracted into FMAs where the compiler chose: u
        # agrees to a few roundoff units; v (c^2 times the Laplacian, with large
        # cancelling terms at the outer cells) to a few hundred relative to its
        # maximum
        assert du <= 1e-13 and dv <= 1e-12
        # the residual is a small difference of much larger Laplacian and
        # source terms, so roundoff-level changes of u move it by ~1e-10
        np.testing.assert_allclose(rr.history, rp.history, rtol=1e-9, atol=1e-16)
        if with_oracle:
            d_or = rel_maxdiff(gr.get_u(extended=True), oracle_extended(og, ou))
            banner(f"resident (8 x {r}) vs oracle: {d_or:.2e}")
            assert d_or <= 1e-12


def test_resident_relaxes_paper_scale_to_tolerance():
    w = workloads.paper_scale()
    banner("resident paper-scale solve to 1e-10")
    g = gpu_grid(w.grid)
    g.set_kernel_config(variant=3)
    g.set_punctures(*w.punctures.as_tuple())
    r = g.relax(w.eta, 1.0, 0.0, 20000, 1e-10, check_every=100)
    h = gpu_grid(w.grid)
    h.set_kernel_config(variant=1)
    h.set_punctures(*w.punctures.as_tuple())
    rp = h.relax(w.eta, 1.0, 0.0, 20000, 1e-10, check_every=100)
    banner(f"resident {r.steps_taken} steps, plane {rp.steps_taken} steps, "
           f"residual {r.residual:.2e}")
    assert r.status == hr.OK and r.steps_taken == rp.steps_taken
    assert g.residual_l2() < 1e-10
    assert rel_maxdiff(g.get_u(extended=True), h.get_u(extended=True)) <= 1e-12


def test_resident_rejected_where_not_applicable():
    for spec in (workloads.GridSpec(0, 37, 19, 6, 10, bscale=1.0),   # not whole patches
                 workloads.GridSpec(0, 32, 16, 4, 6, bscale=1.0),    # order 6
                 workloads.GridSpec(0, 32, 16, 18, 8, bscale=1.0)):  # N2 > 16
        g = gpu_grid(spec)
        with pytest.raises(hr.HRError):
            g.set_kernel_config(variant=3)
    # more patches than compute units (8 x 8 or 8 x 4)
    g = gpu_grid(workloads.GridSpec(0, 256, 256, 8, 10, bscale=1.0))
    with pytest.raises(hr.HRError):
        g.set_kernel_config(variant=3)
    # patch rows other than 4 and 8, and 8-row patches on N1 = 12
    g = gpu_grid(workloads.GridSpec(0, 32, 16, 4, 8, bscale=1.0))
    with pytest.raises(hr.HRError):
        g.set_kernel_config(variant=3, chunk=6)
    g = gpu_grid(workloads.GridSpec(0, 32, 12, 4, 8, bscale=1.0))
    with pytest.raises(hr.HRError):
        g.set_kernel_config(variant=3, chunk=8)
    g.set_kernel_config(variant=3, chunk=4)
    assert g.resolved_kernel(hr.FP64)["chunk"] == 4


def test_resident_stage_timing_keeps_trajectory():
    w = workloads.paper_scale()
    g = gpu_grid(w.grid)
    g.set_kernel_config(variant=3)
    g.set_punctures(*w.punctures.as_tuple())
    t = g.time_stage_kernels(w.eta, 1.0, 0.0, 100, hr.FP64)
    banner(f"resident per-stage time {t[4]:.2f} us")
    assert all(x > 0 for x in t)
    h = gpu_grid(w.grid)
    h.set_kernel_config(variant=1)
    h.set_punctures(*w.punctures.as_tuple())
    h.relax(w.eta, 1.0, 0.0, 100, 0.0, check_every=100)
    assert rel_maxdiff(g.get_u(extended=True), h.get_u(extended=True)) <= 1e-13


@pytest.mark.parametrize("spec", [CASES[0][0], CASES[2][0], CASES[3][0]])
def test_resident_split_form_matches_plane_split_form(spec):
    """The split-state single-precision form (FP32 increment on the FP64 base)
    on the resident kernel against the same form on plane tiles, 300 steps from
    rest with the FP32 phase held: the same FP32 arithmetic per point, rounded
    in a different order, so the two may differ by single-precision rounding of
    the increments (large here: from rest an interval's increment is most of u),
    but the resident form is no further from the FP64 oracle than the plane
    form (within a factor 2) and the two differ by at most twice that
    distance. Near convergence, where the increments are small, the split form
    meets the FP64 solution to 1e-8 (test_gpu_precision)."""
    banner(f"resident split form {spec.name()}")
    og = oracle_grid(spec)
    dt = og.suggest_dt(0.5)
    out = []
    for variant in (3, 1):
        g = gpu_grid(spec)
        g.set_kernel_config(variant=variant)
        g.set_fp32_switch(0.0, 1000000, 0)   # stay in the FP32 phase
        g.set_punctures(*_punctures(spec).as_tuple())
        r = g.relax(6.0, 1.0, dt, 300, 0.0, check_every=100, precision=hr.FP32_FP64FINISH)
        assert r.status == hr.OK and r.fp32_steps == 300
        out.append((g.get_u(extended=True), r.history))
    if spec.N0 == 128:
        assert gpu_grid(spec).resolved_kernel(hr.FP32_FP64FINISH)["variant"] == 3
    og.set_punctures(*_punctures(spec).as_tuple())
    og.relax(6.0, 1.0, dt, 300, 0.0, 100)
    ou, _ = og.state()
    oe = oracle_extended(og, ou)
    d = rel_maxdiff(out[0][0], out[1][0])
    d_res = rel_maxdiff(out[0][0], oe)
    d_pl = rel_maxdiff(out[1][0], oe)
    banner(f"split resident vs split plane {d:.2e}; vs oracle: resident {d_res:.2e}, "
           f"plane {d_pl:.2e}")
    assert d_res <= 2 * d_pl + 1e-12
    assert d <= 2 * d_pl + 1e-12


def test_resident_wait_timeout_falls_back_to_the_stage_kernels():
    """A wait bound of one poll makes the exchange waits give up (a partner is
    rarely done at the first poll), as when the device cannot hold every
    block at once. The kernel's blocks all leave their loops; hr_relax goes
    back to the state it copied before the launch, reruns that interval on the
    stage kernels and stays on them for the rest of the call, counting the
    fallback. The result equals the plane-tile kernels' (same arithmetic), in
    a checked interval and in the unchecked tail, FP64 and split form; with
    the default bound the resident kernel runs again without fallback."""
    w = workloads.paper_scale()
    ref = {}
    for steps in (250, 50):   # two checked intervals and a tail; a tail only
        h = gpu_grid(w.grid)
        h.set_kernel_config(variant=1)
        h.set_punctures(*w.punctures.as_tuple())
        h.relax(w.eta, 1.0, 0.0, steps, 0.0, check_every=100)
        ref[steps] = h.get_u(extended=True)
        h.close()
    g = gpu_grid(w.grid)
    g.set_kernel_config(variant=3)
    g.set_punctures(*w.punctures.as_tuple())
    g.set_wait_limit(1)
    for steps in (250, 50):
        g.set_punctures(*w.punctures.as_tuple())
        r = g.relax(w.eta, 1.0, 0.0, steps, 0.0, check_every=100)
        d = rel_maxdiff(g.get_u(extended=True), ref[steps])
        banner(f"forced wait timeout, {steps} steps: status {r.status}, "
               f"{r.resident_fallbacks} fallback(s), u vs plane tiles {d:.2e}")
        assert r.status == hr.OK and r.steps_taken == steps
        assert r.resident_fallbacks == 1
        assert d <= 1e-13
    g.set_punctures(*w.punctures.as_tuple())
    g.set_fp32_switch(0.0, 8, 0)
    r = g.relax(w.eta, 1.0, 0.0, 60000, w.tol, check_every=100, precision=hr.FP32_FP64FINISH)
    banner(f"split form with the forced timeout: {r.steps_taken} steps, "
           f"{r.resident_fallbacks} fallback(s), residual {r.residual:.2e}")
    assert r.status == hr.OK and r.resident_fallbacks >= 1 and r.residual < w.tol
    g.set_wait_limit(0)
    g.set_punctures(*w.punctures.as_tuple())
    r = g.relax(w.eta, 1.0, 0.0, 250, 0.0, check_every=100)
    assert r.status == hr.OK and r.resident_fallbacks == 0
    assert rel_maxdiff(g.get_u(extended=True), ref[250]) <= 1e-13
