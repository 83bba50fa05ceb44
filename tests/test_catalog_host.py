"""Host logic of the catalog runner: grouping grids so that one batch's
per-stage working set fits the cache budget (no device calls)."""
from types import SimpleNamespace

import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import catalog


def _grids(sizes):
    return [SimpleNamespace(n_extended=n) for n in sizes]


@pytest.mark.parametrize("prec", [hr.FP64, hr.FP32_FP64FINISH])
def test_cache_groups_partition_and_budget(prec):
    big, mid, small = 261 * 256 * 32, 133 * 128 * 16, 69 * 64 * 8
    sizes = [big] * 5 + [mid] * 7 + [small] * 9
    grids = _grids(sizes)
    budget = 200 << 20
    groups = catalog.cache_groups(grids, prec, budget)
    flat = sorted(i for g in groups for i in g)
    assert flat == list(range(len(grids)))            # every grid exactly once
    per = catalog.STAGE_BYTES_PER_POINT["fp64" if prec == hr.FP64 else "split"]
    for g in groups:
        load = sum(sizes[i] * per for i in g)
        assert load <= budget or len(g) == 1          # over budget only when alone
    # FP64: a 256x256x32 grid (~170 MB per stage) never shares its group with
    # another; the split form (~100 MB each) pairs them
    for g in groups:
        assert sum(1 for i in g if sizes[i] == big) <= (1 if prec == hr.FP64 else 2)
    # the small grids fill the remaining room instead of opening new groups
    assert len(groups) <= 5 + 2


def test_cache_groups_unbounded_is_one_batch():
    grids = _grids([1000, 10, 5000])
    assert catalog.cache_groups(grids, hr.FP64, 1 << 62) == [[2, 0, 1]]
