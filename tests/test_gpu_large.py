"""GPU parity at the largest sizes the benchmarks time, in their launch
configurations: the roofline grid SinhSymTP 512x512x64 at 10th order (automatic
choice: phi-column stage kernels, graph-captured check intervals) and a batch
holding a catalog-size 256x256x32 grid with a 128x128x16 one (batched column
kernels). A few RK4 steps keep the oracle within seconds; every stored point
is compared (bar 1e-12 of max|u|, as everywhere in FP64).
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

STEPS, K = 8, 4


def _oracle(spec, pz, eta):
    og = oracle_grid(spec)
    og.set_punctures(*pz.as_tuple())
    dt = og.suggest_dt(0.5)
    st, n, hist = og.relax(eta, 1.0, dt, STEPS, 0.0, K)
    assert st == 0 and n == STEPS
    return og, dt, hist


def test_roofline_grid_512x512x64_parity():
    w = workloads.paper_scale()
    spec = workloads.GridSpec(0, 512, 512, 64, 10, bscale=5.0)
    banner(f"512x512x64 parity, {STEPS} steps")
    og, dt, ohist = _oracle(spec, w.punctures, w.eta)
    ou, ov = og.state()
    g = gpu_grid(spec)
    g.set_punctures(*w.punctures.as_tuple())
    cfg = g.resolved_kernel(hr.FP64)
    res = g.relax(w.eta, 1.0, dt, STEPS, 0.0, check_every=K)
    assert res.status == hr.OK and res.steps_taken == STEPS
    du = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    dv = rel_maxdiff(g.get_v(extended=True), oracle_extended(og, ov))
    banner(f"512x512x64 {cfg}: du {du:.2e} dv {dv:.2e}")
    assert cfg["variant"] == 2
    assert du <= 1e-12 and dv <= 1e-12
    np.testing.assert_allclose(res.history, ohist, rtol=1e-9)
    g.close()


def test_catalog_size_batch_parity():
    banner(f"batch 256x256x32 + 128x128x16 parity, {STEPS} steps")
    pz = workloads.quasi_circular(3.0, 12.0, [0.0, 0.0, 0.4], [0.1, -0.2, 0.0])
    specs = [workloads.GridSpec(0, 256, 256, 32, 10, bscale=6.0),
             workloads.GridSpec(0, 128, 128, 16, 10, bscale=6.0)]
    eta = 80.0
    refs, grids = [], []
    for spec in specs:
        og, _, ohist = _oracle(spec, pz, eta)
        ou, _ = og.state()
        refs.append((oracle_extended(og, ou), ohist))
        g = gpu_grid(spec)
        g.set_punctures(*pz.as_tuple())
        grids.append(g)
    b = hr.Batch(grids)
    try:
        res = b.relax([eta, eta], 1.0, n_steps=STEPS, tol=0.0, check_every=K)
    finally:
        b.close()
    for g, r, (ref, ohist) in zip(grids, res, refs):
        assert r.steps_taken == STEPS
        du = rel_maxdiff(g.get_u(extended=True), ref)
        banner(f"  batch grid {g.N}: du {du:.2e}")
        assert du <= 1e-12
        np.testing.assert_allclose(r.history, ohist, rtol=1e-9)


_PATCH_REF = {}


@pytest.mark.parametrize("n", [1, 3, 7])
def test_independent_patches_batch_parity(n):
    # the independent-patches bench: n identical paper-scale grids in one batch
    # (phi chunks of 2, 4 and 8 planes for n = 1, 3, 7), each against the oracle
    w = workloads.paper_scale()
    spec = w.grid
    banner(f"{n} identical {spec.name()} in one batch, {STEPS} steps")
    if "ref" not in _PATCH_REF:
        og, _, ohist = _oracle(spec, w.punctures, w.eta)
        _PATCH_REF["ref"] = (oracle_extended(og, og.state()[0]), ohist)
    ref, ohist = _PATCH_REF["ref"]
    grids = []
    for _ in range(n):
        g = gpu_grid(spec)
        g.set_punctures(*w.punctures.as_tuple())
        grids.append(g)
    b = hr.Batch(grids)
    try:
        res = b.relax([w.eta] * n, 1.0, n_steps=STEPS, tol=0.0, check_every=K)
    finally:
        b.close()
    u0 = grids[0].get_u(extended=True)
    du = rel_maxdiff(u0, ref)
    banner(f"  du {du:.2e}")
    assert du <= 1e-12
    for g, r in zip(grids, res):
        assert r.steps_taken == STEPS
        assert np.array_equal(g.get_u(extended=True), u0)
        np.testing.assert_allclose(r.history, ohist, rtol=1e-9)
