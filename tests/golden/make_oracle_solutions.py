"""Writes converged oracle solutions, sampled, for the benchmark's larger grids.

Uses the CPU oracle only. For each case it relaxes from u = v = 0 in FP64 until
the residual norm, checked every 100 steps, drops below the tolerance. It
then stores u at a seeded sample of stored points, in the extended layout
(N0 + NG) x N1 x N2 with x0 fastest. The sample always includes the point
where |u| is largest.

The stored values let the benchmark state the error of each of its GPU forms
against the FP64 oracle. That covers FP64, the FP32 bulk with an FP64 finish,
and bfloat16 factors. The oracle's own solve of these grids takes minutes,
too long to repeat inside the benchmark. The paper prints no values for
these grids.

Cases:

* precision-form grids: the equal-mass 32x16x4 physics on 8th-order
  SinhSymTP 128x128x16 (eta 72) and 256x256x32 (eta 290), tolerance 1e-10;
* the paper-scale punctures on the Spherical 128x64x8 grid (10th order,
  rmax 100, eta 2), tolerance 1e-10;
* paper_scale_cartesian_128: the same punctures on the Cartesian cube 128^3,
  [-32, 32]^3, 10th order, eta 0.03, tolerance 1e-10 (the whole padded box is
  the stored layout there; samples are drawn from the evolved points).

Run: python tests/golden/make_oracle_solutions.py [name ...]
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2501_14030_amd import workloads  # noqa: E402  (parameters only)

N_SAMPLE = 4096


def cases():
    return {
        "precision_form_128x128x16": workloads.precision_form(128, 128, 16),
        "precision_form_256x256x32": workloads.precision_form(256, 256, 32),
        "paper_scale_spherical_128x64x8": workloads.paper_scale(workloads.SPHERICAL, 10),
        "paper_scale_cartesian_128": workloads.paper_scale_cartesian(128),
    }


def path_of(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def solve(w):
    s = w.grid
    g = oracle.OracleGrid(s.coords, s.N0, s.N1, s.N2, s.fd_order, amax=s.amax,
                          sinhwaa=s.sinhwaa, bscale=s.bscale, rmax=s.rmax)
    g.set_punctures(*w.punctures.as_tuple())
    dt = g.suggest_dt(w.cfl)
    st, steps, hist = g.relax(w.eta, w.kappa, dt, 200000, w.tol, w.check_every)
    if st != 0:
        raise RuntimeError(f"oracle did not converge: status {st} after {steps} steps")
    u, _ = g.state()
    ng = g.NG
    if s.coords == oracle.CARTESIAN:
        # the library stores the whole padded box; sample only evolved points
        used = (g.bc_images() != -4).reshape(-1)
        return dt, steps, hist, u.reshape(-1), used
    ext = u[ng:ng + s.N2, ng:ng + s.N1, ng:ng + s.N0 + ng].reshape(-1)
    return dt, steps, hist, ext, np.ones(ext.size, dtype=bool)


def write(name: str, w) -> None:
    t0 = time.perf_counter()
    dt, steps, hist, ext, used = solve(w)
    rng = np.random.default_rng(20250124)
    cand = np.flatnonzero(used)
    idx = np.sort(np.unique(np.concatenate(
        [rng.choice(cand, size=N_SAMPLE, replace=False), [int(np.argmax(np.abs(ext)))]])))
    np.savez(path_of(name), idx=idx.astype(np.int64), u=ext[idx], steps=np.int64(steps),
             dt=np.float64(dt), residual_history=hist, max_abs_u=np.float64(np.abs(ext).max()),
             shape=np.array(w.grid.shape, dtype=np.int64), fd_order=np.int64(w.grid.fd_order),
             eta=np.float64(w.eta), tol=np.float64(w.tol))
    print(f"{name}: {steps} steps, residual {hist[-1]:.3e}, {time.perf_counter() - t0:.0f} s "
          f"-> {path_of(name)}", flush=True)


def load(name: str) -> dict:
    with np.load(path_of(name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    all_cases = cases()
    for name in (sys.argv[1:] or list(all_cases)):
        write(name, all_cases[name])
