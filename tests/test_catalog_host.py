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


class _Fake:
    def __init__(self, N, variant, rows, n_ext):
        self.N, self.n_extended = N, n_ext
        self._cfg = {"variant": variant, "chunk": rows, "streaming": 0, "graph": 0}

    def resolved_kernel(self, precision):
        return self._cfg


def test_plan_groups_runs_chip_filling_resident_grids_alone():
    # 128x128x16 on the resident kernel with 8x8 patches: 256 patches, alone on
    # 256 compute units; 64x64x8 (64 patches) and phi-column grids are batched
    big = _Fake((256, 256, 32), 2, 8, 261 * 256 * 32)
    mid = _Fake((128, 128, 16), 3, 8, 133 * 128 * 16)
    mid4 = _Fake((128, 64, 16), 3, 4, 133 * 64 * 16)      # 16 x 16 patches of 8 x 4
    small = _Fake((64, 64, 8), 3, 8, 69 * 64 * 8)
    grids = [small, mid, big, small, mid, mid4]
    assert catalog.runs_alone(mid, hr.FP64, 256)
    assert catalog.runs_alone(mid4, hr.FP64, 256)
    assert not catalog.runs_alone(mid, hr.FP64, 304)
    assert not catalog.runs_alone(small, hr.FP64, 256)
    assert not catalog.runs_alone(big, hr.FP64, 256)
    groups = catalog.plan_groups(grids, hr.FP64, 200 << 20, 256)
    assert groups[:3] == [[1], [4], [5]]
    assert sorted(i for g in groups for i in g) == list(range(len(grids)))
    assert sorted(sorted(g) for g in groups[3:]) == sorted(
        sorted([[0, 2, 3][j] for j in grp])
        for grp in catalog.cache_groups([small, big, small], hr.FP64, 200 << 20))
