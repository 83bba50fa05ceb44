"""The stage-kernel variants (plane tiles; phi-marching columns with a
register queue) and the cache-policy switch compute the same arithmetic in
the same order: their trajectories must agree with each other (to a few
roundoff units) and with the oracle, including ragged phi chunks. The
automatic choice, the autotuner (which may pick the resident kernel, tested
on its own in test_gpu_resident) and graph capture are checked here too."""
import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

from gpu_common import banner, gpu_grid, oracle_extended, oracle_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

CASES = [
    (workloads.GridSpec(0, 32, 16, 4, 8, bscale=1.0), 3),
    (workloads.GridSpec(0, 37, 19, 6, 10, bscale=1.0), 4),
    (workloads.GridSpec(1, 33, 18, 10, 8, rmax=50.0), 3),
    (workloads.GridSpec(0, 70, 20, 2, 10, amax=100.0, sinhwaa=0.2, bscale=1.0), 1),
]


def _relax(spec, pz, cfg, n_steps, dt):
    g = gpu_grid(spec)
    g.set_kernel_config(**cfg)
    g.set_punctures(*pz.as_tuple())
    res = g.relax(6.0, 1.0, dt, n_steps, 0.0, check_every=100)
    assert res.status == hr.OK
    return g.get_u(extended=True), g.get_v(extended=True), res.history


@pytest.mark.parametrize("spec,chunk", CASES)
def test_column_variant_matches_oracle_and_plane_variant(spec, chunk):
    banner(f"variants {spec.name()} chunk {chunk}")
    pz = workloads.quasi_circular(2.3, 2 * spec.bscale if spec.coords == 0 else 8.0,
                                  [0.0, 0.3, 0.1], [0.2, 0.0, -0.3])
    og = oracle_grid(spec)
    og.set_punctures(*pz.as_tuple())
    dt = og.suggest_dt(0.5)
    og.relax(6.0, 1.0, dt, 300, 0.0, 100)
    ou, _ = og.state()
    up, vp, hp = _relax(spec, pz, dict(variant=1, streaming=0), 300, dt)
    uc, vc, hc = _relax(spec, pz, dict(variant=2, streaming=0, chunk=chunk), 300, dt)
    un, vn, hn = _relax(spec, pz, dict(variant=1, streaming=1), 300, dt)
    d_or = rel_maxdiff(uc, oracle_extended(og, ou))
    d_pc = rel_maxdiff(uc, up)
    banner(f"column vs oracle {d_or:.2e}, column vs plane {d_pc:.2e}")
    assert d_or <= 1e-12
    assert d_pc <= 1e-14 and rel_maxdiff(vc, vp) <= 1e-14
    np.testing.assert_allclose(hc, hp, rtol=1e-12, atol=1e-16)
    # the cache-policy switch changes nothing numerically
    assert np.array_equal(un, up) and np.array_equal(vn, vp)


def test_automatic_variant_choice_on_paper_scale():
    w = workloads.paper_scale()
    g = gpu_grid(w.grid)
    cfg = g.kernel_config()
    assert cfg["variant"] == 0 and cfg["streaming"] == -1
    # automatic: the resident kernel for FP64 at this size, plane tiles for FP32
    assert g.resolved_kernel(hr.FP64)["variant"] == 3
    assert g.resolved_kernel(hr.FP32)["variant"] == 1
    g.set_kernel_config(variant=2, streaming=0, chunk=0)
    g.set_punctures(*w.punctures.as_tuple())
    r = g.relax(w.eta, 1.0, 0.0, 100, 0.0, check_every=100)
    uc = g.get_u(extended=True)
    g.set_kernel_config(variant=1, streaming=0, chunk=0)
    g.set_punctures(*w.punctures.as_tuple())
    g.relax(w.eta, 1.0, 0.0, 100, 0.0, check_every=100)
    assert rel_maxdiff(uc, g.get_u(extended=True)) <= 1e-14
    assert r.status == hr.OK


def test_invalid_kernel_config_rejected():
    w = workloads.equal_mass_small()
    g = gpu_grid(w.grid)
    with pytest.raises(hr.HRError):
        g.set_kernel_config(variant=5)
    with pytest.raises(hr.HRError):
        g.set_kernel_config(variant=2, chunk=-1)


def test_autotune_keeps_state_and_caches():
    banner("autotune")
    w = workloads.paper_scale()
    spec = workloads.GridSpec(0, 64, 64, 16, 10, bscale=5.0)
    g = gpu_grid(spec)
    g.set_punctures(*w.punctures.as_tuple())
    g.relax(16.0, 1.0, 0.0, 100, 0.0, check_every=100)
    u0 = g.get_u(extended=True)
    v0 = g.get_v(extended=True)
    cfg, us = g.autotune(hr.FP64, 3)
    assert cfg["variant"] in (1, 2, 3) and us > 0
    if cfg["variant"] == 2:
        assert 1 <= cfg["chunk"] <= spec.N2
    if cfg["variant"] == 3:
        assert cfg["chunk"] in (4, 8)      # resident patch rows
    assert np.array_equal(g.get_u(extended=True), u0)
    assert np.array_equal(g.get_v(extended=True), v0)
    assert g.kernel_config() == cfg
    # a second grid of the same shape takes the cached choice
    h = gpu_grid(spec)
    h.set_punctures(*w.punctures.as_tuple())
    cfg2, us2 = h.autotune(hr.FP64, 3)
    assert cfg2 == cfg and us2 == us
    # the tuned configuration relaxes to the same state as the default one
    g.relax(16.0, 1.0, 0.0, 200, 0.0, check_every=100)
    h.set_kernel_config(variant=1)
    h.set_punctures(*w.punctures.as_tuple())
    h.relax(16.0, 1.0, 0.0, 300, 0.0, check_every=100)
    assert rel_maxdiff(g.get_u(extended=True), h.get_u(extended=True)) <= 1e-13


@pytest.mark.parametrize("prec", [hr.FP64, hr.FP32_FP64FINISH, hr.FP32])
def test_graph_replays_match_eager_launches(prec):
    """Each check interval is one replay of the captured graph; the residual read
    back after every replay and the final state must equal the eager launches'
    bitwise (same kernels, same arguments)."""
    banner(f"graph vs eager, precision {prec}")
    w = workloads.equal_mass_small()
    out = []
    for graph in (0, 1):
        g = gpu_grid(w.grid)
        # plane tiles: the resident kernel (automatic for FP64 here) runs a
        # check interval as one launch and is never captured
        g.set_kernel_config(variant=1, graph=graph)
        g.set_fp32_switch(0.0, 1000000, 0)
        g.set_punctures(*w.punctures.as_tuple())
        r1 = g.relax(8.0, 1.0, 0.0, 700, 0.0, check_every=100, precision=prec)
        # eager host work between replays, then a second call reusing the graph
        _ = g.get_u()
        r2 = g.relax(8.0, 1.0, 0.0, 350, 0.0, check_every=100, precision=prec)
        out.append((np.concatenate([r1.history, r2.history]), g.get_u(extended=True),
                    g.get_v(extended=True)))
    assert len(out[0][0]) == 10
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
