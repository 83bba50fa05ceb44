"""Cartesian grids (the Cartesian-like family the paper's conclusions name)
on the GPU against the oracle.

The cube [-rmax, rmax]^3 stores NG outer layers beyond each of its six faces;
the interior kernel (plane tiles whose rim comes from those layers, z taps
from memory; or z columns with the z taps in a register queue) and the face
kernel (radiation condition along each face normal) update them, in FP64,
FP32 or the split-state form. Bars: FP64 trajectories and converged states
within 1e-12 of the oracle (relative to max|u|, over every stored point),
residual histories to 1e-9 relative; plain FP32 within 1e-4 after 300 steps
(300 steps of single precision rounding, unit roundoff 6e-8, on a state whose
largest value is O(1e-2)); the split form's converged state within 1e-10.
The calls Cartesian grids do not take return HR_EINVAL.
"""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads
from paper_2501_14030_amd.mlp import MLP, config_features

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

CART = workloads.CARTESIAN
SPECS = [
    workloads.GridSpec(CART, 24, 20, 16, 8, rmax=6.0),
    workloads.GridSpec(CART, 70, 13, 11, 10, rmax=5.0),   # ragged tiles, odd sizes
]


def _punct():
    return ([0.5, 0.5], [[0, 0, 1.3], [0, 0, -1.3]],
            [[0, 0.1, 0], [0, -0.1, 0.02]], [[0, 0, 0.1], [0.05, 0, -0.1]])


def _oracle(spec, n_steps, tol, eta, order=2):
    og = oracle_grid(spec)
    if order != 2:
        og.set_bc_order(order)
    og.set_punctures(*_punct())
    st, n, hist = og.relax(eta, 1.0, og.suggest_dt(0.5), n_steps, tol, 100)
    return og, n, hist


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: s.name())
def test_trajectory_matches_oracle(spec):
    eta = 1.0
    og, _, ohist = _oracle(spec, 400, 0.0, eta)
    g = gpu_grid(spec)
    g.set_punctures(*_punct())
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 400, 0.0, check_every=100)
    ou, ov = og.state()
    gu = g.get_u(extended=True)
    assert gu.shape == og.shape
    du = rel_maxdiff(gu, oracle_extended(og, ou))
    dv = rel_maxdiff(g.get_v(extended=True), oracle_extended(og, ov))
    banner(f"{spec.name()}: du {du:.2e} dv {dv:.2e}, history {r.history}")
    assert r.status == hr.OK
    assert du <= 1e-12 and dv <= 1e-12
    np.testing.assert_allclose(r.history, ohist, rtol=1e-9, atol=1e-15)
    # the face layers carry the solution (not zero), the edges stay zero
    img = og.bc_images().reshape(og.shape)
    assert np.abs(gu[img == -2]).max() > 1e-3 * np.abs(gu).max()
    assert np.all(gu[img == -4] == 0.0)


@pytest.mark.parametrize("prec", [hr.FP64, hr.FP32, hr.FP32_FP64FINISH],
                         ids=["fp64", "fp32", "split"])
@pytest.mark.parametrize("chunk", [1, 3, 16])
def test_z_columns_match_plane_tiles_and_oracle(chunk, prec):
    """The interior's column variant (a register queue of z taps, `chunk`
    planes per block; chunk 3 leaves a ragged last chunk of 2 planes on N2 = 11)
    does the plane tiles' arithmetic: the same state bit for bit, and the
    oracle's trajectory in FP64."""
    spec = SPECS[1]
    eta = 1.0
    og, _, ohist = _oracle(spec, 200, 0.0, eta)
    out = []
    for variant in (1, 2):
        g = gpu_grid(spec)
        g.set_kernel_config(variant=variant, chunk=chunk if variant == 2 else 0)
        assert g.resolved_kernel(prec)["variant"] == variant
        g.set_punctures(*_punct())
        r = g.relax(eta, 1.0, og.suggest_dt(0.5), 200, 0.0, check_every=100, precision=prec)
        assert r.status == hr.OK
        out.append((g.get_u(extended=True), g.get_v(extended=True), r.history))
    (u1, v1, h1), (u2, v2, h2) = out
    banner(f"z columns, chunk {chunk}, precision {prec}: max |u_col - u_tiles| "
           f"{np.abs(u2 - u1).max():.2e}")
    assert np.array_equal(u1, u2) and np.array_equal(v1, v2)
    assert list(h1) == list(h2)
    if prec == hr.FP64:
        ou, _ = og.state()
        assert rel_maxdiff(u2, oracle_extended(og, ou)) <= 1e-12
        np.testing.assert_allclose(h2, ohist, rtol=1e-9, atol=1e-15)


def test_paper_scale_cube_runs_on_z_columns():
    """The 128^3 cube resolves to the column variant (chunk 8), and 20 steps on
    it equal 20 steps on the plane tiles bit for bit."""
    w = workloads.paper_scale_cartesian()
    states = []
    for cfg in ({}, {"variant": 1}):
        g = gpu_grid(w.grid)
        if cfg:
            g.set_kernel_config(**cfg)
        else:
            rk = g.resolved_kernel(hr.FP64)
            assert rk["variant"] == 2 and rk["chunk"] == 8
        g.set_punctures(*w.punctures.as_tuple())
        r = g.relax(w.eta, 1.0, 0.0, 20, 0.0, check_every=10)
        assert r.status == hr.OK
        states.append(g.get_u(extended=True))
        g.close()
    assert np.array_equal(states[0], states[1])


def test_converged_state_matches_oracle():
    spec = SPECS[0]
    eta = 1.0
    og, n_or, _ = _oracle(spec, 200000, 1e-10, eta)
    ou, _ = og.state()
    g = gpu_grid(spec)
    g.set_punctures(*_punct())
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 200000, 1e-10, check_every=100)
    du = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    banner(f"{spec.name()} to 1e-10: {r.steps_taken} steps (oracle {n_or}), du {du:.2e}")
    assert r.status == hr.OK and r.steps_taken == n_or and du <= 1e-12
    # the allocation-free entry point runs the same kernels
    g.set_punctures(*_punct())
    rn = g.relax_noalloc(eta, 1.0, og.suggest_dt(0.5), 200000, 1e-10, check_every=100)
    assert rn.status == hr.OK and rn.steps_taken == n_or
    assert rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou)) <= 1e-12


def test_fourth_order_faces_match_oracle():
    spec = SPECS[0]
    eta = 1.0
    og, _, ohist = _oracle(spec, 300, 0.0, eta, order=4)
    g = gpu_grid(spec)
    g.set_outer_bc_order(4)
    g.set_punctures(*_punct())
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 300, 0.0, check_every=100)
    ou, _ = og.state()
    du = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    banner(f"order-4 faces: du {du:.2e}")
    assert du <= 1e-12
    np.testing.assert_allclose(r.history, ohist, rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("bits,bound", [(32, 1e-10), (16, 1e-9)])
def test_split_form_converges_to_oracle_state(bits, bound):
    """The split-state form (FP32 increment on an FP64 base re-evaluated every
    check, FP64 finish below ten times the tolerance) on the Cartesian grid:
    the interior and face kernels' single-precision increment, the base
    slopes of both, and the rebase. Bars as for the curvilinear grids: the
    state converged to 1e-10 within 1e-10 of the oracle's converged state
    (relative to max|u|; 1e-9 with bfloat16 factors), at least half of the
    steps in FP32."""
    spec = SPECS[0]
    eta = 1.0
    og, n_or, _ = _oracle(spec, 200000, 1e-10, eta)
    ou, _ = og.state()
    g = gpu_grid(spec)
    g.set_fp32_switch(0.0, 8, 0)
    g.set_factor_storage(bits)
    g.set_punctures(*_punct())
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 200000, 1e-10, check_every=100,
                precision=hr.FP32_FP64FINISH)
    du = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    banner(f"split form, {bits}-bit factors: {r.steps_taken} steps ({r.fp32_steps} fp32; "
           f"oracle {n_or}), du vs oracle {du:.2e}")
    assert r.status == hr.OK and g.residual_l2() < 1e-10
    assert du <= bound
    assert r.fp32_steps >= 0.5 * r.steps_taken
    img = og.bc_images().reshape(og.shape)
    assert np.all(g.get_u(extended=True)[img == -4] == 0.0)


def test_fp32_state_tracks_oracle():
    spec = SPECS[0]
    eta = 1.0
    og, _, _ = _oracle(spec, 300, 0.0, eta)
    g = gpu_grid(spec)
    g.set_punctures(*_punct())
    r = g.relax(eta, 1.0, og.suggest_dt(0.5), 300, 0.0, check_every=100, precision=hr.FP32)
    ou, _ = og.state()
    du = rel_maxdiff(g.get_u(extended=True), oracle_extended(og, ou))
    banner(f"FP32 state after 300 steps: du {du:.2e}")
    assert r.status == hr.OK and du <= 1e-4


def test_interior_set_u_continues_faces_as_one_over_r():
    spec = SPECS[0]
    g = gpu_grid(spec)
    g.set_punctures(*_punct())
    og = oracle_grid(spec)
    X, Y, Z = og.cart()
    R = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    ng, (N0, N1, N2) = og.NG, og.N
    f = 1.0 / R   # its continuation from each face's adjacent interior layer is itself
    g.set_u(og.interior(f))
    got = g.get_u(extended=True)
    img = og.bc_images().reshape(og.shape)
    np.testing.assert_allclose(got[img == -1], f[img == -1], rtol=0, atol=0)
    np.testing.assert_allclose(got[img == -2], f[img == -2], rtol=1e-14, atol=0)
    assert np.all(got[img == -4] == 0.0)


def test_calls_cartesian_grids_do_not_take():
    spec = SPECS[0]
    g = gpu_grid(spec)
    g.set_punctures(*_punct())
    with pytest.raises(hr.HRError) as e:
        g.set_residual_norm(hr.NORM_VOLUME)
    assert e.value.status == hr.EINVAL
    with pytest.raises(hr.HRError) as e:
        hr.Batch([g])
    assert e.value.status == hr.EINVAL
    net = MLP(width=16, seed=1, max_batch=4096)
    with pytest.raises(hr.HRError) as e:
        net.warm_start(g, config_features(1.0, [0, 0, 0], [0, 0, 0], 0.1, 2.6), 1.0)
    assert e.value.status == hr.EINVAL
    net.close()
    assert g.resolved_kernel(hr.FP64)["variant"] == 1
    # the grid still relaxes after the refusals
    r = g.relax(1.0, 1.0, 0.0, 100, 0.0, check_every=50)
    assert r.status == hr.OK and np.isfinite(r.residual)
