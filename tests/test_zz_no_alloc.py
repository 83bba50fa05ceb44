"""hr_relax_noalloc (the FP64 relaxation whose scratch lives in the library's
static device array) against hr_relax on the same inputs, through the C ABI.

Two calls in a row, the second on a smaller grid, so that the second runs on
scratch that still holds the first call's contents:
* SinhSymTP 128x128x16, 10th order (the resident kernel), to residual 1e-10;
* a ragged SinhSymTP 37x19x6, 10th order (the stage kernels), 600 steps.
Both kernels take the same inputs, so the bar is the parity bar of the FP64
form (max|du|/max|u| <= 1e-12); equal step counts and residual histories too.
Then hr_relax continues on the grid that ran hr_relax_noalloc (its workspace
pointers restored), and the size limit and the loaded-c rule are checked.
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, rel_maxdiff

pytestmark = pytest.mark.gpu


def _pair(spec, punct):
    a, b = gpu_grid(spec), gpu_grid(spec)
    for g in (a, b):
        g.set_punctures(*punct.as_tuple())
    return a, b


def _compare(a, b, ra, rb, label):
    du = rel_maxdiff(b.get_u(extended=True), a.get_u(extended=True))
    dv = rel_maxdiff(b.get_v(extended=True), a.get_v(extended=True))
    banner(f"{label}: hr_relax {ra.steps_taken} steps, noalloc {rb.steps_taken}; "
           f"du {du:.2e} dv {dv:.2e}")
    assert ra.status == rb.status == hr.OK
    assert ra.steps_taken == rb.steps_taken
    assert du <= 1e-12 and dv <= 1e-12
    np.testing.assert_allclose(rb.history, ra.history, rtol=1e-12, atol=0)


def test_noalloc_matches_relax_on_two_calls_in_a_row():
    w = workloads.paper_scale(workloads.SINHSYMTP, 10)
    a, b = _pair(w.grid, w.punctures)
    assert a.resolved_kernel(hr.FP64)["variant"] == 3
    dt = a.suggest_dt(w.cfl)
    ra = a.relax(w.eta, w.kappa, dt, 20000, w.tol, check_every=w.check_every)
    rb = b.relax_noalloc(w.eta, w.kappa, dt, 20000, w.tol, check_every=w.check_every)
    _compare(a, b, ra, rb, f"{w.grid.name()} (resident kernel)")
    assert rb.residual < w.tol

    small = workloads.GridSpec(workloads.SINHSYMTP, 37, 19, 6, 10, bscale=1.0)
    c0 = workloads.equal_mass_small()
    a2, b2 = _pair(small, c0.punctures)
    assert a2.resolved_kernel(hr.FP64)["variant"] in (1, 2)
    dt2 = a2.suggest_dt(0.5)
    ra = a2.relax(1.0, 1.0, dt2, 600, 0.0, check_every=100)
    rb = b2.relax_noalloc(1.0, 1.0, dt2, 600, 0.0, check_every=100)
    _compare(a2, b2, ra, rb, f"{small.name()} (stage kernels)")

    # hr_relax on the grid that ran hr_relax_noalloc: the workspace is intact
    ra = a2.relax(1.0, 1.0, dt2, 300, 0.0, check_every=100)
    rb = b2.relax(1.0, 1.0, dt2, 300, 0.0, check_every=100)
    _compare(a2, b2, ra, rb, f"{small.name()} continued with hr_relax")


def test_noalloc_limits():
    w = workloads.paper_scale(workloads.SINHSYMTP, 10)
    big = workloads.GridSpec(workloads.SINHSYMTP, 256, 256, 32, 10, bscale=w.grid.bscale)
    g = gpu_grid(big)
    g.set_punctures(*w.punctures.as_tuple())
    with pytest.raises(hr.HRError) as ei:
        g.relax_noalloc(w.eta, 1.0, 0.0, 4, 0.0, check_every=4)
    assert ei.value.status == hr.ENOMEM
    g.close()
    small = workloads.GridSpec(workloads.SINHSYMTP, 37, 19, 6, 10, bscale=1.0)
    g = gpu_grid(small)
    g.set_punctures(*workloads.equal_mass_small().punctures.as_tuple())
    with pytest.raises(hr.HRError) as ei:
        g.relax_noalloc(1.0, 2.0, 0.0, 4, 0.0, check_every=4)
    assert ei.value.status == hr.ESTATE
    g.relax(1.0, 2.0, 0.0, 4, 0.0, check_every=4)   # loads c = 2
    r = g.relax_noalloc(1.0, 2.0, 0.0, 4, 0.0, check_every=4)
    assert r.status == hr.OK and r.steps_taken == 4
