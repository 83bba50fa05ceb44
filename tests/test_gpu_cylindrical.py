"""SinhCylindrical (the cylindrical-like family the paper's conclusions name)
on the GPU against the oracle.

The stored layout keeps NG outer rows beyond each z face; the stage kernels
(plane tiles and phi columns, also inside a batch) update them with the
radiation condition, taking the one-sided difference along xx1 where
|z| >= rho and along xx0 elsewhere. The resident kernel does not take these
grids. Bars as for the other families: FP64 trajectories and converged states
within 1e-12 of the oracle (relative to max|u|, over every stored point, the
z-face rows included); the split single-precision form within 2e-8 at
convergence on this coarse grid (measured 9.1e-9: its 1600 FP32 steps take
dt = 0.029, so the last FP32 increments, whose single-precision rounding the
FP64 finish inherits, are large next to u; on the paper-scale grids the same
form stays below 1e-9).
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

CYL = workloads.SINHCYLINDRICAL
SPECS = [
    workloads.GridSpec(CYL, 32, 16, 4, 8, amax=10.0, sinhwaa=0.3),
    workloads.GridSpec(CYL, 37, 22, 6, 10, amax=1.0e3, sinhwaa=0.15),   # ragged tiles
]


def _punct(k=0):
    return ([0.5, 0.5], [[0, 0, 1.0], [0, 0, -1.0]],
            [[0, 0.1 + 0.05 * k, 0], [0, -0.1, 0.02]], [[0, 0, 0.1], [0.05, 0, -0.1]])


def _oracle(spec, n_steps, tol, eta, order=2):
    og = oracle_grid(spec)
    if order != 2:
        og.set_bc_order(order)
    og.set_punctures(*_punct())
    st, n, hist = og.relax(eta, 1.0, og.suggest_dt(0.5), n_steps, tol, 100)
    return og, n, hist


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: s.name())
@pytest.mark.parametrize("kernel", [{"variant": 1}, {"variant": 2, "chunk": 2}],
                         ids=["plane", "columns"])
def test_trajectory_matches_oracle(spec, kernel):
    eta = 2.0
    og, _, ohist = _oracle(spec, 600, 0.0, eta)
    g = gpu_grid(spec)
    g.set_kernel_config(**kernel)
    g.set_punctures(*_punct())
    assert g.resolved_kernel(hr.FP64)["variant"] != 3
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 600, 0.0, check_every=100)
    ou, ov = og.state()
    du = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    dv = rel_maxdiff(g.get_v(extended=True), oracle_extended(og, ov))
    banner(f"{spec.name()} {kernel}: du {du:.2e} dv {dv:.2e}")
    assert r.status == hr.OK
    assert du <= 1e-12 and dv <= 1e-12
    np.testing.assert_allclose(r.history, ohist, rtol=1e-9, atol=1e-13)


def test_converged_state_and_split_form_match_oracle():
    spec = SPECS[0]
    eta = 2.0
    og, n_or, _ = _oracle(spec, 200000, 1e-10, eta)
    ou, _ = og.state()
    ref = oracle_extended(og, ou)
    g = gpu_grid(spec)
    g.set_punctures(*_punct())
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 200000, 1e-10, check_every=100)
    du = rel_maxdiff(g.get_u(extended=True), ref)
    banner(f"{spec.name()} to 1e-10: {r.steps_taken} steps (oracle {n_or}), du {du:.2e}")
    assert r.status == hr.OK and r.steps_taken == n_or and du <= 1e-12
    g.set_punctures(*_punct())
    g.set_fp32_switch(0.0, 8, 0)
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 200000, 1e-10, check_every=100,
                precision=hr.FP32_FP64FINISH)
    du = rel_maxdiff(g.get_u(extended=True), ref)
    banner(f"  split form: {r.steps_taken} steps ({r.fp32_steps} fp32), du {du:.2e}")
    assert r.status == hr.OK and r.fp32_steps > 0 and du <= 2e-8


def test_fourth_order_outer_condition_matches_oracle():
    spec = SPECS[1]
    eta = 2.0
    og, _, _ = _oracle(spec, 400, 0.0, eta, order=4)
    ou, _ = og.state()
    for kernel in ({"variant": 1}, {"variant": 2, "chunk": 2}):
        g = gpu_grid(spec)
        g.set_kernel_config(**kernel)
        g.set_outer_bc_order(4)
        g.set_punctures(*_punct())
        g.relax(eta, 1.0, og.suggest_dt(0.5), 400, 0.0, check_every=100)
        du = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
        banner(f"{spec.name()} outer order 4 {kernel}: du {du:.2e}")
        assert du <= 1e-12


def test_cylindrical_grid_in_a_batch():
    specs = [SPECS[1], workloads.GridSpec(0, 37, 19, 6, 10, bscale=3.0)]
    pz = [_punct(1), workloads.quasi_circular(1.5, 6.0, [0.1, 0, 0.2], [0, -0.1, 0.1])]
    gs = []
    for spec, p in zip(specs, pz):
        g = gpu_grid(spec)
        g.set_punctures(*(p if isinstance(p, tuple) else p.as_tuple()))
        gs.append(g)
    b = hr.Batch(gs)
    res = b.relax([2.0, 4.0], 1.0, n_steps=500, tol=0.0, check_every=100)
    assert b.status == hr.OK
    for spec, p, g, eta, rb in zip(specs, pz, gs, [2.0, 4.0], res):
        e = gpu_grid(spec)
        e.set_punctures(*(p if isinstance(p, tuple) else p.as_tuple()))
        r = e.relax(eta, 1.0, 0.0, 500, 0.0, check_every=100)
        d = rel_maxdiff(g.get_u(extended=True), e.get_u(extended=True))
        banner(f"  {spec.name()} batch vs eager {d:.2e}")
        assert d <= 1e-13
        np.testing.assert_allclose(rb.history, r.history, rtol=1e-9, atol=1e-16)
