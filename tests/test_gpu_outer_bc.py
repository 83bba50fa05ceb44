"""GPU parity of the fourth-order one-sided difference in the outer radiation
condition (hr_set_outer_bc_order(g, 4)) against the oracle with the same
option, for every kernel that applies the condition: plane tiles, phi
columns, the resident kernel, the split-state FP32 form (its FP64 base slopes
and FP32 increment stages) and a batch. Bar: the FP64 parity bar, 1e-12 of
max|u|, at equal step counts; the split form against its own plane-tile
result to the distance the plain split form keeps (it is FP32 arithmetic).
The order-4 trajectory must differ from the order-2 one (the option takes
effect), and its outer slopes are pinned on the oracle side.
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

SPECS = [
    (workloads.GridSpec(0, 32, 16, 4, 8, bscale=1.0), "SinhSymTP 32x16x4 order 8"),
    (workloads.GridSpec(0, 37, 19, 6, 10, bscale=1.0), "ragged SinhSymTP order 10"),
    (workloads.GridSpec(1, 64, 32, 8, 10, rmax=100.0), "Spherical 64x32x8 order 10"),
    (workloads.GridSpec(2, 64, 32, 8, 8), "SinhSpherical 64x32x8 order 8"),
]
PZ = workloads.quasi_circular(1.7, 2.0, [0.0, 0.2, 0.3], [0.1, 0.0, -0.2])
ETA, STEPS = 6.0, 400


def _oracle(spec, order, steps=STEPS):
    og = oracle_grid(spec)
    og.set_bc_order(order)
    og.set_punctures(*PZ.as_tuple())
    dt = og.suggest_dt(0.5)
    og.relax(ETA, 1.0, dt, steps, 0.0, 100)
    return og, dt


def _gpu(spec, order, dt, steps=STEPS, precision=hr.FP64, **cfg):
    g = gpu_grid(spec)
    g.set_outer_bc_order(order)
    if cfg:
        g.set_kernel_config(**cfg)
    g.set_punctures(*PZ.as_tuple())
    res = g.relax(ETA, 1.0, dt, steps, 0.0, check_every=100, precision=precision)
    assert res.status == hr.OK and res.steps_taken == steps
    return g, res


@pytest.mark.parametrize("spec,label", SPECS)
def test_fourth_order_outer_bc_parity_every_kernel(spec, label):
    banner(f"outer bc order 4 {label}")
    og, dt = _oracle(spec, 4)
    ou, ov = og.state()
    ref = oracle_extended(og, ou)
    kinds = [dict(variant=1), dict(variant=2, chunk=2)]
    g0 = gpu_grid(spec)
    if g0.resolved_kernel(hr.FP64)["variant"] == 3:
        kinds.append(dict(variant=3))
    for cfg in kinds:
        g, _ = _gpu(spec, 4, dt, **cfg)
        d = rel_maxdiff(g.get_u(extended=True), ref)
        dv = rel_maxdiff(g.get_v(extended=True), oracle_extended(og, ov))
        banner(f"  {cfg}: du {d:.2e} dv {dv:.2e}")
        assert d <= 1e-12 and dv <= 1e-12
    # the option takes effect: order 2 gives another trajectory near the boundary
    og2, _ = _oracle(spec, 2)
    u2 = oracle_extended(og2, og2.state()[0])
    assert rel_maxdiff(u2, ref) > 1e-9


@pytest.mark.parametrize("spec,label", [SPECS[0], SPECS[2]])
def test_fourth_order_outer_bc_split_form(spec, label):
    banner(f"outer bc order 4, split form {label}")
    og, dt = _oracle(spec, 4)
    ref = oracle_extended(og, og.state()[0])
    gp, _ = _gpu(spec, 4, dt, precision=hr.FP32_FP64FINISH, variant=1)
    d_plane = rel_maxdiff(gp.get_u(extended=True), ref)
    g2p, _ = _gpu(spec, 2, dt, precision=hr.FP32_FP64FINISH, variant=1)
    og2, _ = _oracle(spec, 2)
    d_plane2 = rel_maxdiff(g2p.get_u(extended=True), oracle_extended(og2, og2.state()[0]))
    banner(f"  split plane vs oracle: order 4 {d_plane:.2e}, order 2 {d_plane2:.2e}")
    # FP32 increments: the order-4 form stays as close as the order-2 form
    assert d_plane <= 2 * d_plane2 + 1e-12
    g0 = gpu_grid(spec)
    if g0.resolved_kernel(hr.FP32_FP64FINISH)["variant"] == 3:
        gr, _ = _gpu(spec, 4, dt, precision=hr.FP32_FP64FINISH, variant=3)
        d_res = rel_maxdiff(gr.get_u(extended=True), ref)
        banner(f"  split resident vs oracle {d_res:.2e}")
        assert d_res <= 2 * d_plane + 1e-12


def test_fourth_order_outer_bc_in_a_batch():
    banner("outer bc orders 4 and 2 in one batch")
    # each grid keeps its own order inside a batch
    specs = [(SPECS[1][0], 4), (SPECS[2][0], 2)]
    refs, grids, dts = [], [], []
    for spec, order in specs:
        og, dt = _oracle(spec, order)
        refs.append(oracle_extended(og, og.state()[0]))
        g = gpu_grid(spec)
        g.set_outer_bc_order(order)
        g.set_punctures(*PZ.as_tuple())
        grids.append(g)
        dts.append(dt)
    b = hr.Batch(grids)
    try:
        res = b.relax([ETA, ETA], 1.0, n_steps=STEPS, tol=0.0, check_every=100)
    finally:
        b.close()
    for g, r, ref in zip(grids, res, refs):
        assert r.steps_taken == STEPS
        d = rel_maxdiff(g.get_u(extended=True), ref)
        banner(f"  batch grid du {d:.2e}")
        assert d <= 1e-12


def test_outer_bc_order_errors():
    g = gpu_grid(SPECS[0][0])
    for bad in (1, 3, 6):
        with pytest.raises(hr.HRError):
            g.set_outer_bc_order(bad)
