"""Batched relaxation (one persistent launch per RK stage over many grids,
graph-captured per check interval) against the same grids relaxed one at a
time with the eager single-grid path.

Every check interval replays the captured graph; the per-grid residual
histories compared below check every replay against the eager result, and the
final states are compared point by point. The batch uses the phi-column
kernel body for every grid, the eager path may use plane tiles: both evaluate
the same arithmetic in the same order, so results agree to a few roundoff
units. FP64 results are also compared with the CPU oracle.
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

SPECS = [
    workloads.GridSpec(0, 37, 19, 6, 10, bscale=3.0),
    workloads.GridSpec(0, 64, 64, 8, 10, bscale=4.0),
    workloads.GridSpec(1, 40, 24, 4, 10, rmax=60.0),
    workloads.GridSpec(0, 20, 12, 2, 10, amax=100.0, sinhwaa=0.2, bscale=2.0),
]


def _punctures(spec, k):
    D = 2 * spec.bscale if spec.coords == 0 else 10.0
    return workloads.quasi_circular(1.0 + 0.7 * k, D, [0.1 * k, 0.0, 0.2], [0.0, -0.1, 0.1 * k])


def _grids():
    gs = []
    for k, spec in enumerate(SPECS):
        g = gpu_grid(spec)
        g.set_punctures(*_punctures(spec, k).as_tuple())
        gs.append(g)
    return gs


def test_batch_fixed_steps_matches_eager_and_oracle():
    banner("batch fixed steps")
    etas = [4.0, 8.0, 6.0, 5.0]
    gs = _grids()
    b = hr.Batch(gs)
    res = b.relax(etas, 1.0, n_steps=300, tol=0.0, check_every=100)
    assert b.status == hr.OK
    for k, spec in enumerate(SPECS):
        e = gpu_grid(spec)
        e.set_punctures(*_punctures(spec, k).as_tuple())
        r = e.relax(etas[k], 1.0, 0.0, 300, 0.0, check_every=100)
        d = rel_maxdiff(gs[k].get_u(extended=True), e.get_u(extended=True))
        banner(f"{spec.name()}: batch vs eager {d:.2e}")
        assert d <= 1e-13
        # the residual is a small difference of much larger terms: roundoff-level
        # differences of u (column kernels here, the resident kernel eagerly) move
        # it by up to ~1e-10 relative
        np.testing.assert_allclose(res[k].history, r.history, rtol=1e-9, atol=1e-16)
        assert res[k].steps_taken == 300
    # one grid against the oracle as well
    spec = SPECS[0]
    og = oracle_grid(spec)
    og.set_punctures(*_punctures(spec, 0).as_tuple())
    og.relax(etas[0], 1.0, og.suggest_dt(0.5), 300, 0.0, 100)
    ou, _ = og.state()
    assert rel_maxdiff(gs[0].get_u(extended=True), oracle_extended(og, ou)) <= 1e-12


@pytest.mark.parametrize("prec", [hr.FP64, hr.FP32_FP64FINISH])
def test_batch_to_tolerance_each_grid_stops_on_its_own(prec):
    banner(f"batch to tolerance prec {prec}")
    etas = [4.0, 8.0, 6.0, 5.0]
    gs = _grids()
    b = hr.Batch(gs)
    res = b.relax(etas, 1.0, n_steps=60000, tol=1e-10, check_every=100, precision=prec)
    assert b.status == hr.OK
    for k, spec in enumerate(SPECS):
        e = gpu_grid(spec)
        e.set_punctures(*_punctures(spec, k).as_tuple())
        r = e.relax(etas[k], 1.0, 0.0, 60000, 1e-10, check_every=100, precision=prec)
        assert r.status == hr.OK
        banner(f"{spec.name()}: batch steps {res[k].steps_taken} (fp32 {res[k].fp32_steps}), "
               f"eager {r.steps_taken} (fp32 {r.fp32_steps})")
        assert res[k].steps_taken == r.steps_taken
        assert res[k].fp32_steps == r.fp32_steps
        assert gs[k].residual_l2() < 1e-10
        assert rel_maxdiff(gs[k].get_u(extended=True), e.get_u(extended=True)) <= 1e-11


def test_batch_rejects_mixed_orders_and_unbound():
    a = gpu_grid(workloads.GridSpec(0, 16, 8, 2, 8, bscale=1.0))
    c = gpu_grid(workloads.GridSpec(0, 16, 8, 2, 10, bscale=1.0))
    with pytest.raises(hr.HRError):
        hr.Batch([a, c])
    with pytest.raises(hr.HRError):
        hr.Batch([a, a])


def test_identical_grids_in_one_batch_and_batch_reuse():
    # the independent-patches setup of Sec. 4: N identical grids in one batch
    # relax exactly alike (no cross-talk between work-list entries), match one
    # eager solve, and a batch relaxed a second time from u = v = 0 repeats itself
    banner("identical grids in one batch, reused")
    spec = workloads.GridSpec(0, 64, 64, 8, 10, bscale=4.0)
    pz = _punctures(spec, 1)
    gs = [gpu_grid(spec) for _ in range(5)]
    for g in gs:
        g.set_punctures(*pz.as_tuple())
    b = hr.Batch(gs)
    res = b.relax([6.0] * 5, 1.0, n_steps=60000, tol=1e-10, check_every=100)
    u0 = gs[0].get_u(extended=True)
    for g, r in zip(gs, res):
        assert r.status == hr.OK and r.steps_taken == res[0].steps_taken
        assert np.array_equal(g.get_u(extended=True), u0)
        np.testing.assert_array_equal(r.history, res[0].history)
    e = gpu_grid(spec)
    e.set_punctures(*pz.as_tuple())
    r = e.relax(6.0, 1.0, 0.0, 60000, 1e-10, check_every=100)
    banner(f"  batch steps {res[0].steps_taken}, eager {r.steps_taken}")
    assert r.steps_taken == res[0].steps_taken
    assert rel_maxdiff(u0, e.get_u(extended=True)) <= 1e-11
    for g in gs:
        g.set_punctures(*pz.as_tuple())
    res2 = b.relax([6.0] * 5, 1.0, n_steps=60000, tol=1e-10, check_every=100)
    b.close()
    for g, r in zip(gs, res2):
        assert r.steps_taken == res[0].steps_taken
        assert np.array_equal(g.get_u(extended=True), u0)


def test_batch_phi_chunks_with_ragged_tails():
    # two 128x128x14 grids and one 128x128x10: the batch walks phi in chunks of
    # 4 planes (352 work items), so each column ends on a ragged chunk (2 planes)
    banner("batch phi chunks of 4 with ragged tails")
    specs = [workloads.GridSpec(0, 128, 128, 14, 10, bscale=4.0),
             workloads.GridSpec(0, 128, 128, 14, 10, bscale=5.0),
             workloads.GridSpec(0, 128, 128, 10, 10, bscale=4.0)]
    etas = [20.0, 30.0, 25.0]
    gs = []
    for k, spec in enumerate(specs):
        g = gpu_grid(spec)
        g.set_punctures(*_punctures(spec, k).as_tuple())
        gs.append(g)
    b = hr.Batch(gs)
    res = b.relax(etas, 1.0, n_steps=200, tol=0.0, check_every=100)
    b.close()
    for k, spec in enumerate(specs):
        assert res[k].steps_taken == 200
        e = gpu_grid(spec)
        e.set_punctures(*_punctures(spec, k).as_tuple())
        r = e.relax(etas[k], 1.0, 0.0, 200, 0.0, check_every=100)
        d = rel_maxdiff(gs[k].get_u(extended=True), e.get_u(extended=True))
        banner(f"  {spec.name()}: batch vs eager {d:.2e}")
        assert d <= 1e-13
        np.testing.assert_allclose(res[k].history, r.history, rtol=1e-9, atol=1e-16)
    spec = specs[2]
    og = oracle_grid(spec)
    og.set_punctures(*_punctures(spec, 2).as_tuple())
    og.relax(etas[2], 1.0, og.suggest_dt(0.5), 200, 0.0, 100)
    ou, _ = og.state()
    assert rel_maxdiff(gs[2].get_u(extended=True), oracle_extended(og, ou)) <= 1e-12


def test_batch_reports_a_non_finite_grid():
    """A grid whose wave speed breaks the RK4 stability limit (kappa 50, local
    Courant number 25) blows up inside a batch: the batch returns
    HR_ENONFINITE, that grid's result says so, and the other grid keeps
    relaxing to its step cap (HR_ENOTCONV under an unreachable tolerance)."""
    banner("batch with one unstable grid")
    spec = workloads.GridSpec(0, 32, 16, 4, 8, bscale=1.0)
    pz = workloads.equal_mass_small().punctures
    gs = [gpu_grid(spec) for _ in range(2)]
    for g in gs:
        g.set_punctures(*pz.as_tuple())
    b = hr.Batch(gs)
    res = b.relax([1.0, 1.0], [1.0, 50.0], n_steps=1000, tol=1e-30, check_every=100,
                  raise_on_error=False)
    b.close()
    banner(f"  status {b.status}, grids {[r.status for r in res]}, "
           f"residuals {[r.residual for r in res]}")
    assert b.status == hr.ENONFINITE
    assert res[1].status == hr.ENONFINITE
    assert res[0].status == hr.ENOTCONV and res[0].steps_taken == 1000
    assert np.isfinite(res[0].residual)


# Grids small enough for the resident kernel share resident launches inside a
# batch: five 64x64x8 grids (64 patches of 8 x 8 each) and two 48x32x6 grids
# (24 each) take the same kernel instance (10th order, up to 8 planes), so
# they pack into launches of at most one patch per compute unit; a ragged
# grid stays on the batched stage kernels. Each grid keeps its own counters
# and exchange buffers, so every result must equal its eager single-grid
# solve (the resident and the stage kernels evaluate the same arithmetic in
# the same order), and the first grid is compared with the oracle as well.
SMALL = [workloads.GridSpec(0, 64, 64, 8, 10, bscale=1.0 + 0.5 * k) for k in range(5)] + \
        [workloads.GridSpec(0, 48, 32, 6, 10, bscale=2.0), workloads.GridSpec(0, 48, 32, 6, 10, bscale=3.0),
         workloads.GridSpec(0, 37, 19, 6, 10, bscale=3.0)]


@pytest.mark.parametrize("prec", [hr.FP64, hr.FP32_FP64FINISH])
def test_small_grids_share_resident_launches(prec):
    banner(f"small grids in shared resident launches, prec {prec}")
    gs = []
    etas = []
    for k, spec in enumerate(SMALL):
        g = gpu_grid(spec)
        g.set_punctures(*_punctures(spec, k).as_tuple())
        gs.append(g)
        etas.append(workloads.eta_for_dt(g.suggest_dt(0.5)))
    b = hr.Batch(gs)
    res = b.relax(etas, 1.0, n_steps=60000, tol=1e-10, check_every=100, precision=prec)
    assert b.status == hr.OK
    for k, spec in enumerate(SMALL):
        e = gpu_grid(spec)
        e.set_punctures(*_punctures(spec, k).as_tuple())
        if prec == hr.FP32_FP64FINISH:
            e.set_fp32_switch(0.0, 8, 0)
        r = e.relax(etas[k], 1.0, 0.0, 60000, 1e-10, check_every=100, precision=prec)
        d = rel_maxdiff(gs[k].get_u(extended=True), e.get_u(extended=True))
        banner(f"  {spec.name()}: batch {res[k].steps_taken} steps ({res[k].fp32_steps} fp32), "
               f"eager {r.steps_taken} ({r.fp32_steps}); u {d:.2e}")
        assert res[k].steps_taken == r.steps_taken and res[k].fp32_steps == r.fp32_steps
        assert d <= (1e-13 if prec == hr.FP64 else 1e-12)
        np.testing.assert_allclose(res[k].history, r.history, rtol=1e-9, atol=1e-13)
        e.close()
    if prec == hr.FP64:
        spec = SMALL[0]
        og = oracle_grid(spec)
        og.set_punctures(*_punctures(spec, 0).as_tuple())
        og.relax(etas[0], 1.0, og.suggest_dt(0.5), res[0].steps_taken, 0.0, 100)
        ou, _ = og.state()
        d = rel_maxdiff(gs[0].get_u(extended=True), oracle_extended(og, ou))
        banner(f"  {spec.name()} vs oracle after {res[0].steps_taken} steps: {d:.2e}")
        assert d <= 1e-12
    b.close()
