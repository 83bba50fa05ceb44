"""Relaxation of a catalog of independent configurations on one GPU.

The batched path (``Batch``: one persistent launch per RK stage over every grid
in the batch) is grouped so that the grid functions one stage touches stay
within the Infinity Cache: MI355X has 256 MB of it in front of HBM, and a
256x256x32 grid alone touches ~170 MB per FP64 stage. Batching all the large
grids of a catalog together streams every stage from HBM; relaxing them in
cache-sized groups lets each stage re-read what the previous one wrote from the
cache. Grids are placed largest first into the first group with room (a grid
larger than the budget gets a group of its own).

A grid whose own kernel is the resident one with a patch on every compute unit
(128x128x16 and larger (x0, x1) planes that fit it) is relaxed alone instead:
the resident kernel keeps its state on chip and already fills the chip, which
no batch of stage kernels matches (3.2 us per stage alone against ~7 us per
grid and stage in a batch at 128x128x16, FP64).
"""
from __future__ import annotations

import time

import numpy as np

from . import FP64, Batch

# bytes per stored point that one RK stage touches: FP64 state y_n, two stage
# buffers, accumulator (u and v each), psi_s and S_src; the split-state form
# reads the same set in FP32 plus the base slopes, p_b and S_src p_b^-7
STAGE_BYTES_PER_POINT = {"fp64": 10 * 8, "split": 12 * 4}
CACHE_BUDGET = 200 << 20


def cache_groups(grids, precision: int, budget: int = CACHE_BUDGET) -> list:
    """Index groups of `grids` whose per-stage working sets add up to at most
    `budget` bytes (first fit, largest grids first)."""
    per = STAGE_BYTES_PER_POINT["fp64" if precision == FP64 else "split"]
    order = sorted(range(len(grids)), key=lambda i: -grids[i].n_extended)
    groups, loads = [], []
    for i in order:
        need = grids[i].n_extended * per
        for k, load in enumerate(loads):
            if load + need <= budget:
                groups[k].append(i)
                loads[k] += need
                break
        else:
            groups.append([i])
            loads.append(need)
    return groups


def runs_alone(g, precision: int, cus: int) -> bool:
    """True if `g` relaxes faster by itself: its automatic kernel in this
    precision is the resident kernel and its patches (8 x0 points by `chunk`
    x1 rows) cover at least `cus` compute units."""
    cfg = g.resolved_kernel(precision)
    if cfg["variant"] != 3:
        return False
    N0, N1, _ = g.N
    return (N0 // 8) * (N1 // cfg["chunk"]) >= cus


def plan_groups(grids, precision: int, budget: int = CACHE_BUDGET, cus: int = 256) -> list:
    """Index groups in the order they are relaxed: each grid that runs alone
    (`runs_alone`), then the cache groups of the others."""
    solo = [i for i, g in enumerate(grids) if runs_alone(g, precision, cus)]
    taken = set(solo)
    rest = [i for i in range(len(grids)) if i not in taken]
    sub = cache_groups([grids[i] for i in rest], precision, budget)
    return [[i] for i in solo] + [[rest[j] for j in grp] for grp in sub]


def autotune_batches(ws, grids, precision: int, groups, etas, steps: int = 40, log=None) -> dict:
    """Batch-level tile tuning for the groups that run as batches. The members
    of a group whose own kernel is not the resident one go through the batched
    phi-column stage body; for each distinct composition of such members (their
    sorted shapes) a batch of fresh grids of the same configurations (`ws`) is
    timed at every phi chunk 1, 2, 4, ... up to their largest N2 (`steps` RK4
    steps after one untimed pass that captures the interval's graph), and the
    fastest chunk is set on the members as an explicit phi-column
    configuration, which the batch keeps. Returns {composition: (chunk,
    {chunk: seconds})}; the catalog's own grids are not stepped."""
    import torch

    from .warmstart import make_grids

    tuned = {}
    for group in groups:
        if len(group) < 2:
            continue
        members = [i for i in group if grids[i].resolved_kernel(precision)["variant"] != 3]
        if not members:
            continue
        key = tuple(sorted(tuple(grids[i].N) for i in members))
        if key not in tuned:
            fresh = make_grids([ws[i] for i in members], None)
            times = {}
            c = 1
            while c <= max(g.N[2] for g in fresh):
                for g in fresh:
                    g.set_kernel_config(variant=2, chunk=min(c, g.N[2]))
                b = Batch(fresh)
                e = [etas[i] for i in members]
                b.relax(e, 1.0, n_steps=steps, tol=0.0, check_every=steps, precision=precision,
                        raise_on_error=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.relax(e, 1.0, n_steps=steps, tol=0.0, check_every=steps, precision=precision,
                        raise_on_error=False)
                torch.cuda.synchronize()
                times[c] = time.perf_counter() - t0
                b.close()
                c *= 2
            for g in fresh:
                g.close()
            best = min(times, key=times.get)
            tuned[key] = (best, times)
            if log:
                log(f"batch tuning {key}: chunk {best} "
                    f"({', '.join(f'{k}: {v * 1e3:.1f} ms' for k, v in times.items())})")
        for i in members:
            grids[i].set_kernel_config(variant=2, chunk=min(tuned[key][0], grids[i].N[2]))
    return tuned


def relax_catalog(grids, etas, tols, precision: int = FP64, max_steps: int = 60000,
                  chunk: int = 5000, check_every: int = 100, budget: int = CACHE_BUDGET,
                  log=None):
    """Relaxes every grid to its own tolerance with its own eta. Returns (steps
    taken, last residual) per grid. Each cache group of several grids is relaxed
    in chunks of `chunk` steps (one batched call per tolerance within the group),
    a grid leaving its batch at its first check below its tolerance; a group of
    one grid is relaxed by the single-grid path."""
    import torch

    steps = [0] * len(grids)
    resid = [float("inf")] * len(grids)
    t0 = time.perf_counter()
    if not grids:
        return steps, resid
    cus = torch.cuda.get_device_properties(grids[0].device).multi_processor_count
    groups = plan_groups(grids, precision, budget, cus)
    for gi, group in enumerate(groups):
        if len(group) == 1:
            # a grid alone: the single-grid path (same kernels, no work lists)
            i = group[0]
            r = grids[i].relax(etas[i], 1.0, 0.0, max_steps, tols[i], check_every=check_every,
                               precision=precision, raise_on_error=False)
            steps[i], resid[i] = r.steps_taken, r.residual
            if log:
                log(f"catalog group {gi + 1}/{len(groups)} (1 grid) done after "
                    f"{time.perf_counter() - t0:.1f} s")
            continue
        active = list(group)
        while active and max(steps[i] for i in active) < max_steps:
            nxt = []
            for tol in sorted(set(tols[i] for i in active)):
                sub = [i for i in active if tols[i] == tol]
                b = Batch([grids[i] for i in sub])
                res = b.relax([etas[i] for i in sub], 1.0, n_steps=chunk, tol=tol,
                              check_every=check_every, precision=precision,
                              raise_on_error=False)
                b.close()
                for i, r in zip(sub, res):
                    steps[i] += r.steps_taken
                    resid[i] = r.residual
                    if not (r.residual < tol) and np.isfinite(r.residual):
                        nxt.append(i)
            active = sorted(nxt)
        if log:
            log(f"catalog group {gi + 1}/{len(groups)} ({len(group)} grids) done after "
                f"{time.perf_counter() - t0:.1f} s")
    return steps, resid


def warm_start_catalog(mlp, ws, grids, etas, smooth=None) -> int:
    """Learned warm start of every catalog grid before its relaxation: the
    network's prediction of u on each grid (inference kernels; v = m eta u),
    the smoothing phase of warmstart.SMOOTH batched over all grids, then
    v = eta u. The relaxation that follows still decides convergence. Returns
    the smoothing steps each grid took."""
    from . import warmstart

    smooth = warmstart.SMOOTH if smooth is None else smooth
    m, ns = smooth
    for w, g, e in zip(ws, grids, etas):
        mlp.warm_start(g, warmstart.config_of(w), m * e if ns > 0 else e)
    return warmstart.smooth_all(grids, etas, smooth)
