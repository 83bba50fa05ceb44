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
