"""Single-precision forms against FP64 (paper: single-precision builds,
"Roofline Analysis" subsection; here the bulk steps run in FP32 while the
residual norm, the stop test and the final phase stay in FP64).

Stated errors (checked below):
* split-state FP32 bulk (HR_FP32_FP64FINISH), fixed 1000 steps of the 32x16x4
  case: max|u - u_oracle| / max|u_oracle| <= 1e-8;
* the same form relaxed to residual 1e-10: max|u - u_fp64| / max|u_fp64| <= 1e-8
  against the FP64 form relaxed to the same tolerance, with the FP64 residual
  of the result below the tolerance and most steps taken in FP32;
* plain FP32 state (HR_FP32), 1000 steps: <= 1e-4 (its residual floor is set by
  single precision).
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu


def _oracle_config0(n_steps):
    w = workloads.equal_mass_small()
    og = oracle_grid(w.grid)
    og.set_punctures(*w.punctures.as_tuple())
    dt = og.suggest_dt(w.cfl)
    og.relax(w.eta, 1.0, dt, n_steps, 0.0, w.check_every)
    return w, og, dt


def test_split_fp32_trajectory_close_to_oracle():
    w, og, dt = _oracle_config0(1000)
    ou, _ = og.state()
    g = gpu_grid(w.grid)
    g.set_fp32_switch(0.0, 1000000, 0)  # never leave the single-precision phase
    g.set_punctures(*w.punctures.as_tuple())
    r = g.relax(w.eta, 1.0, dt, 1000, 0.0, check_every=100, precision=hr.FP32_FP64FINISH)
    assert r.status == hr.OK and r.fp32_steps == 1000
    d = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    banner(f"split FP32 1000 steps: rel diff vs oracle {d:.2e}")
    assert d <= 1e-8


def test_plain_fp32_trajectory_error_bound():
    w, og, dt = _oracle_config0(1000)
    ou, _ = og.state()
    g = gpu_grid(w.grid)
    g.set_punctures(*w.punctures.as_tuple())
    r = g.relax(w.eta, 1.0, dt, 1000, 0.0, check_every=100, precision=hr.FP32)
    assert r.status == hr.OK and r.fp32_steps == 1000
    d = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    banner(f"plain FP32 1000 steps: rel diff vs oracle {d:.2e}")
    assert d <= 1e-4


@pytest.mark.parametrize("spec", [workloads.GridSpec(0, 64, 64, 8, 10, bscale=5.0),
                                  workloads.GridSpec(0, 128, 128, 16, 10, bscale=5.0)])
def test_split_fp32_converges_to_fp64_solution(spec):
    w = workloads.paper_scale()
    eta = 16.0 if spec.N0 == 64 else w.eta
    g = gpu_grid(spec)
    g.set_punctures(*w.punctures.as_tuple())
    r64 = g.relax(eta, 1.0, 0.0, 200000, 1e-10, check_every=100, precision=hr.FP64)
    u64 = g.get_u(extended=True)
    g.set_punctures(*w.punctures.as_tuple())
    r32 = g.relax(eta, 1.0, 0.0, 200000, 1e-10, check_every=100, precision=hr.FP32_FP64FINISH)
    u32 = g.get_u(extended=True)
    d = rel_maxdiff(u32, u64)
    banner(f"{spec.name()}: fp64 {r64.steps_taken} steps, split {r32.steps_taken} "
           f"({r32.fp32_steps} fp32), rel diff {d:.2e}, residual {r32.residual:.2e}")
    assert r64.status == hr.OK and r32.status == hr.OK
    assert g.residual_l2() < 1e-10
    assert d <= 1e-8
    assert r32.fp32_steps >= 0.8 * r32.steps_taken


def test_bfloat16_factor_storage():
    """16-bit (bfloat16) storage of the metric factors read by the single-
    precision stages. Stated errors: the split form with these factors, relaxed
    to residual 1e-10 on the 8th-order 128x128x16 precision-form grid, stays
    within 1e-8 of the FP64 solution (the FP64 rebase and finish remove the
    factor rounding from the fixed point); the plain FP32 trajectory moves by
    the factor rounding (between 1e-6 and 1e-2 of max|u| after 1000 steps); the
    FP64 form does not read them (bitwise unchanged)."""
    w = workloads.precision_form(128, 128, 16)
    eta = 80.0
    g = gpu_grid(w.grid)
    g.set_punctures(*w.punctures.as_tuple())
    r64 = g.relax(eta, 1.0, 0.0, 200000, 1e-10, check_every=100, precision=hr.FP64)
    u64 = g.get_u(extended=True)
    g.set_factor_storage(16)
    g.set_punctures(*w.punctures.as_tuple())
    r64b = g.relax(eta, 1.0, 0.0, 200000, 1e-10, check_every=100, precision=hr.FP64)
    assert np.array_equal(g.get_u(extended=True), u64) and r64b.steps_taken == r64.steps_taken
    g.set_punctures(*w.punctures.as_tuple())
    r16 = g.relax(eta, 1.0, 0.0, 200000, 1e-10, check_every=100, precision=hr.FP32_FP64FINISH)
    d16 = rel_maxdiff(g.get_u(extended=True), u64)
    banner(f"bf16 factors, split form: {r16.steps_taken} steps ({r16.fp32_steps} fp32), "
           f"rel diff vs fp64 {d16:.2e}, residual {r16.residual:.2e} (fp64: {r64.steps_taken})")
    assert r16.status == hr.OK and g.residual_l2() < 1e-10
    assert d16 <= 1e-8
    # plain FP32 with 32- and 16-bit factors
    g.set_punctures(*w.punctures.as_tuple())
    g.relax(eta, 1.0, 0.0, 1000, 0.0, check_every=100, precision=hr.FP32)
    ub = g.get_u(extended=True)
    g.set_factor_storage(32)
    g.set_punctures(*w.punctures.as_tuple())
    g.relax(eta, 1.0, 0.0, 1000, 0.0, check_every=100, precision=hr.FP32)
    uf = g.get_u(extended=True)
    dpl = rel_maxdiff(ub, uf)
    banner(f"plain FP32, bf16 vs fp32 factors after 1000 steps: {dpl:.2e}")
    assert 1e-6 < dpl < 1e-2
