"""The catalog runner on the GPU: a small mixed catalog (one grid whose
resident kernel has a patch on every compute unit, relaxed alone, and smaller
grids in cache groups, one of them under a budget that splits the groups)
relaxed to its tolerances in FP64 and in the split form, against the same
grids relaxed one at a time by the single-grid path: equal step counts, every
grid below its tolerance, states within the batch-vs-eager bar."""
import numpy as np
import pytest
import torch

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import catalog, workloads

from gpu_common import banner, gpu_grid, rel_maxdiff

pytestmark = pytest.mark.gpu

SPECS = [
    workloads.GridSpec(0, 128, 128, 4, 10, bscale=4.0),
    workloads.GridSpec(0, 32, 32, 4, 10, bscale=3.0),
    workloads.GridSpec(0, 48, 24, 6, 10, bscale=3.0),
    workloads.GridSpec(1, 40, 24, 4, 10, rmax=60.0),
]


ETAS = [None, 6.0, 5.0, 6.0]   # None: eta_for_dt (the catalog's own rule)


def _pz(k):
    spec = SPECS[k]
    D = 2 * spec.bscale if spec.coords == 0 else 10.0
    return workloads.quasi_circular(1.0 + 0.5 * k, D, [0.0, 0.1 * k, 0.2], [0.1, 0.0, -0.1 * k])


def _make():
    gs = []
    for k, spec in enumerate(SPECS):
        g = gpu_grid(spec)
        g.set_punctures(*_pz(k).as_tuple())
        gs.append(g)
    return gs


@pytest.mark.parametrize("prec", [hr.FP64, hr.FP32_FP64FINISH])
def test_catalog_runner_matches_single_grid_solves(prec):
    banner(f"catalog runner, precision {prec}")
    gs = _make()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    etas = [e if e else workloads.eta_for_dt(g.suggest_dt(0.5)) for e, g in zip(ETAS, gs)]
    tols = [1e-10] * len(gs)
    # a budget that holds the two SinhSymTP side grids but not the Spherical one too
    per = catalog.STAGE_BYTES_PER_POINT["fp64" if prec == hr.FP64 else "split"]
    budget = (gs[1].n_extended + gs[2].n_extended) * per
    groups = catalog.plan_groups(gs, prec, budget, cus)
    banner(f"  groups {groups}")
    if cus <= 256 and gs[0].resolved_kernel(prec)["variant"] == 3:
        assert groups[0] == [0]
    assert sorted(i for g in groups for i in g) == list(range(len(gs)))
    steps, resid = catalog.relax_catalog(gs, etas, tols, prec, max_steps=60000, budget=budget)
    for k, spec in enumerate(SPECS):
        e = gpu_grid(spec)
        e.set_punctures(*_pz(k).as_tuple())
        r = e.relax(etas[k], 1.0, 0.0, 60000, tols[k], check_every=100, precision=prec)
        banner(f"  {spec.name()}: catalog {steps[k]} steps, eager {r.steps_taken}")
        assert r.status == hr.OK
        assert steps[k] == r.steps_taken
        assert resid[k] < tols[k]
        assert rel_maxdiff(gs[k].get_u(extended=True), e.get_u(extended=True)) <= 1e-11
        assert np.isfinite(resid[k])


def test_batch_tile_tuner_sets_a_measured_chunk():
    """catalog.autotune_batches times a batched composition at every phi
    chunk on fresh grids and sets the fastest on the members (an explicit
    phi-column configuration); the catalog's own grids are not stepped, and a
    catalog run with the tuned chunk still matches the eager solves."""
    banner("batch tile tuner")
    specs = [workloads.GridSpec(0, 64, 64, 32, 10, bscale=4.0),
             workloads.GridSpec(0, 48, 32, 24, 10, bscale=3.0)]
    ws = [workloads.Workload(s, workloads.quasi_circular(1.5, 2 * s.bscale, [0, 0, 0.2],
                                                         [0.1, 0, 0]),
                             eta=6.0, label=f"tuner[{k}]") for k, s in enumerate(specs)]
    gs = []
    for w in ws:
        g = gpu_grid(w.grid)
        g.set_punctures(*w.punctures.as_tuple())
        gs.append(g)
    etas = [workloads.eta_for_dt(g.suggest_dt(0.5)) for g in gs]
    tuned = catalog.autotune_batches(ws, gs, hr.FP64, [[0, 1]], etas, steps=20, log=banner)
    (key, (chunk, times)), = tuned.items()
    assert sorted(times) == [1, 2, 4, 8, 16, 32] and chunk == min(times, key=times.get)
    for g in gs:
        cfg = g.kernel_config()
        assert cfg["variant"] == 2 and cfg["chunk"] == min(chunk, g.N[2])
        assert np.all(g.get_u() == 0.0)   # not stepped
    steps, resid = catalog.relax_catalog(gs, etas, [1e-10, 1e-10], hr.FP64, max_steps=60000,
                                         budget=1 << 40)
    for k, w in enumerate(ws):
        e = gpu_grid(w.grid)
        e.set_punctures(*w.punctures.as_tuple())
        r = e.relax(etas[k], 1.0, 0.0, 60000, 1e-10, check_every=100)
        assert steps[k] == r.steps_taken and resid[k] < 1e-10
        assert rel_maxdiff(gs[k].get_u(extended=True), e.get_u(extended=True)) <= 1e-11
