"""Helpers shared by the GPU tests: run the same seeded workload through the
HIP library (via its C ABI binding) and through the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads


def banner(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def oracle_grid(spec: workloads.GridSpec) -> oracle.OracleGrid:
    return oracle.OracleGrid(spec.coords, spec.N0, spec.N1, spec.N2, spec.fd_order,
                             amax=spec.amax, sinhwaa=spec.sinhwaa, bscale=spec.bscale,
                             rmax=spec.rmax)


def gpu_grid(spec: workloads.GridSpec) -> hr.Grid:
    p = hr.default_params(amax=spec.amax, sinhwaa=spec.sinhwaa, bscale=spec.bscale,
                          rmax=spec.rmax)
    return hr.grid_create(spec.coords, spec.N0, spec.N1, spec.N2, spec.fd_order, params=p)


def oracle_extended(g: oracle.OracleGrid, f: np.ndarray) -> np.ndarray:
    """Interior + outer points of a padded oracle field, in the library's
    extended layout (N2, N1, N0 + NG); SinhCylindrical also keeps the NG outer
    rows beyond each z face (N2, N1 + 2 NG, N0 + NG); Cartesian keeps the whole
    padded box (its unused edge and corner points are zero on both sides)."""
    ng = g.NG
    N0, N1, N2 = g.N
    if g.coords == oracle.CARTESIAN:   # every stored point: the padded box
        return np.asarray(f).reshape(g.shape)
    rows = slice(0, N1 + 2 * ng) if g.coords == oracle.SINHCYLINDRICAL else slice(ng, ng + N1)
    return np.asarray(f).reshape(g.shape)[ng:ng + N2, rows, ng:ng + N0 + ng]


def rel_maxdiff(a: np.ndarray, b: np.ndarray) -> float:
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))
