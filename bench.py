"""Benchmark of the hyperbolic-relaxation hot path on one MI355X.

One "step" of this benchmark is one whole solve of the paper-scale workload:
set the punctures (sources on the device, u = v = 0) and relax with RK4 until
the residual L2 norm drops below 1e-10, residual checked every 100 steps. The
workload is the paper's production configuration: SinhSymTP 128x128x16,
10th-order finite differences, equal-mass punctures at z = +-5 with momenta
+-0.095 y_hat and spins (0,0,0.2), synthetic parameters (no dataset involved).

Printed: one JSON line. ``value`` is grid-point RHS updates per second of the
FP64 form over the timed solves (N_interior x 4 RK stages x RK4 steps / wall
time). The FP32-bulk + FP64-finish form and the wall time to residual 1e-10
are reported beside it, with the stage-kernel roofline and the CPU oracle on
the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("grid-pt RHS updates/sec (FP64 vs FP32+FP64 finish); wall time to residual 1e-10")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6    # MI355X vector FP64
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32
GOLDEN = os.path.join(ROOT, "tests", "golden")


def flops_per_update(fd_order: int) -> int:
    """Algorithmic floating-point operations of one grid-point RHS update (one
    fused RK4 stage at one interior point), NG = fd_order / 2 taps a side:
    second-derivative sums 3 x (3 NG + 2), first-derivative sums 2 x 3 NG, the
    five-term Laplacian 9, the source (psi + u)^-7 S with one division 6, the
    two right-hand sides 4, the stage combine 7 (mean over the four stages).
    107 at 10th order, 92 at 8th."""
    ng = fd_order // 2
    return 3 * (3 * ng + 2) + 2 * 3 * ng + 9 + 6 + 4 + 7
KERNEL_SRCS = [os.path.join(ROOT, "paper_2501_14030_amd", "csrc", f)
               for f in ("hr_kernels.hip", "hr_resident.hip", "hr_stencil.h")]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "stage_kernel_pmc.json")


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(shape, prec: str, variant: int = 0, cart: bool = False):
    """Per-launch HBM bytes (mean over the four stage kernels) from the committed
    rocprofv3 PMC summary, if it was taken on the current kernel source; FETCH_SIZE
    and WRITE_SIZE are scaled by what they read for a plain copy of known size."""
    try:
        with open(PMC_SUMMARY) as f:
            pmc = json.load(f)
    except (OSError, ValueError):
        return None
    if pmc.get("kernel_sha") != kernel_sha():
        return None
    key = (f"{shape[0]}x{shape[1]}x{shape[2]}_{prec}" + ("_resident" if variant == 3 else "") +
           ("_cartesian" if cart else ""))
    ent = pmc.get("runs", {}).get(key)
    if not ent:
        return None
    ff = pmc["calibration"]["fetch_factor"]
    wf = pmc["calibration"]["write_factor"]
    per = [1024.0 * (ff * fk + wf * wk) for fk, wk in zip(ent["fetch_kib"], ent["write_kib"])]
    return sum(per) / len(per)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes_per_point(itemsize: int, split: bool = False):
    """Algorithmic bytes per point of the four fused stage kernels.

    interior point: stage 1 reads u, v, psi, S_src and writes Y2(u,v), acc(u,v);
    stages 2, 3 read Y(u,v), y_n(u,v), acc(u,v), psi, S_src and write Y(u,v),
    acc(u,v); stage 4 reads Y4(u,v), acc(u,v), psi, S_src and writes y_{n+1}(u,v).
    outer point: the same without psi and S_src. The split-state form's
    increment stages also read the base slopes k(y_b) (two values; p_b and
    S_src p_b^-7 take the places of psi and S_src).
    """
    extra = 2 if split else 0
    interior = [8 + extra, 12 + extra, 12 + extra, 8 + extra]
    outer = [6 + extra, 10 + extra, 10 + extra, 6 + extra]
    return [itemsize * n for n in interior], [itemsize * n for n in outer]


def stage_algorithmic_bytes(spec, itemsize: int, split: bool = False, cart: bool = False):
    """Per-launch algorithmic bytes of each stage kernel (grid functions plus the
    2D coefficient tables, each read once). Cartesian grids (cart): interior
    kernel and face kernel together, NG face layers beyond each of the six faces
    (their coordinates come from three short tables, not counted)."""
    N0, N1, N2 = spec.shape
    ng = spec.fd_order // 2
    nint = N0 * N1 * N2
    bi, bo = stage_bytes_per_point(itemsize, split)
    if cart:
        nface = 2 * ng * (N1 * N2 + N0 * N2 + N0 * N1)
        return [nint * bi[s] + nface * bo[s] + itemsize * 6 * N0 * N1 for s in range(4)]
    nout = ng * N1 * N2
    tables = itemsize * (6 * N0 * N1 + 3 * ng * N1)
    return [nint * bi[s] + nout * bo[s] + tables for s in range(4)]


VARIANT_NAMES = {1: "fused RK4 stage kernel, plane tiles",
                 2: "fused RK4 stage kernel, phi columns",
                 3: "resident RK4 kernel (whole steps per launch, state on chip)"}


def roofline_entry(g, hr, spec, w, prec, nsteps=20):
    """Roofline of the dominant kernel on the HBM bound: algorithmic bytes of the
    RK4 stages over their mean duration. Stage kernels are timed with HIP events
    recorded in each kernel's own dispatch; the resident kernel runs all 4 x
    nsteps stages in one launch, timed the same way, and each stage is charged
    the launch duration / (4 nsteps). Algorithmic bytes are those a fused stage
    must move when the state lives in HBM (the resident kernel keeps it on chip,
    so its rate may exceed what HBM alone would allow)."""
    item = 8 if prec == hr.FP64 else 4
    split = prec == hr.FP32_FP64FINISH
    cfg = g.resolved_kernel(prec)
    if cfg["variant"] == 3:
        nsteps = w.check_every   # the launch length the relaxation itself uses
    us = g.time_stage_kernels(w.eta, w.kappa, 0.0, nsteps, prec)
    byts = stage_algorithmic_bytes(spec, item, split)
    agg = sum(byts) / (sum(us[:4]) * 1e-6) / 1e9
    pname = "FP64" if prec == hr.FP64 else ("FP32 split-state increment" if split else "FP32")
    tr = None if split else measured_traffic(spec.shape, "fp64" if prec == hr.FP64 else "fp32",
                                             cfg["variant"])
    out = {
        "bound": "hbm", "achieved": agg, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": agg / HBM_PEAK_GBS, "traffic": tr,
        "kernel": f"{VARIANT_NAMES[cfg['variant']]} ({pname}, "
                  f"order {spec.fd_order}, {spec.N0}x{spec.N1}x{spec.N2}, config {cfg}), "
                  f"mean over stages 1-4",
        "avg_stage_us": [float(x) for x in us[:4]],
        "algorithmic_bytes_per_stage": byts,
        "algorithmic_bytes_mean": sum(byts) / 4,
        "traffic_over_algorithmic": (tr / (sum(byts) / 4)) if tr else None,
    }
    if cfg["variant"] == 3:
        out["stages_per_launch"] = 4 * nsteps
        out["avg_launch_us"] = float(us[4]) * 4 * nsteps
    else:
        out["stages_per_launch"] = 1
        out["avg_launch_us"] = [float(x) for x in us[:4]]
    return out


def pmc_summary():
    """The committed rocprofv3 PMC summary if it was taken on the current kernel
    sources, else None."""
    try:
        with open(PMC_SUMMARY) as f:
            pmc = json.load(f)
    except (OSError, ValueError):
        return None
    return pmc if pmc.get("kernel_sha") == kernel_sha() else None


def resident_roofline(hr, spec, prec, timing):
    """Roofline entry of the resident RK4 kernel, timed on the launches of the
    timed solves themselves (HIP events inside each dispatch, on the grid's
    stream). The kernel keeps the whole state in registers and LDS, so HBM does
    not bound it; the entry is placed on the vector-ALU roof of its precision
    (algorithmic flops per launch over the mean launch duration), with the
    measured HBM counter traffic, LDS activity and the rate a fused stage kernel
    streaming the state through HBM would need beside it."""
    fp64 = prec == hr.FP64
    nl = max(1, timing["launches"])
    avg_us = timing["total_us"] / nl
    stages = timing["stages"] / nl
    n_int = spec.n_interior
    fpu = flops_per_update(spec.fd_order)
    flops = fpu * n_int * stages
    achieved = flops / (avg_us * 1e-6) / 1e12
    peak = FP64_PEAK_TFLOPS if fp64 else FP32_PEAK_TFLOPS
    item = 8 if fp64 else 4
    # bytes a fused stage kernel must move per interior point (mean of the four
    # stages' 8, 12, 12, 8 values) if the state lived in HBM
    stream_bytes = item * 10 * n_int * stages
    out = {
        "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
        "frac": achieved / peak, "traffic": None,
        "kernel": f"resident RK4 kernel ({'FP64' if fp64 else 'FP32 split-state increment'}, "
                  f"order {spec.fd_order}, {spec.N0}x{spec.N1}x{spec.N2}), launches of the timed "
                  f"solves",
        "launches_timed": timing["launches"], "stages_per_launch": stages,
        "avg_launch_us": avg_us, "avg_stage_us": avg_us / stages,
        "flops_per_update": fpu, "algorithmic_flops_per_launch": flops,
        "limiter": "latency of the per-stage patch exchange (publish, counter, rim load) plus "
                   "LDS-bound stencil work; neither HBM nor the vector ALU is saturated",
        "as_if_streamed": {"bytes_per_update": item * 10,
                           "gbs": stream_bytes / (avg_us * 1e-6) / 1e9,
                           "frac_of_hbm_peak": stream_bytes / (avg_us * 1e-6) / 1e9 /
                                               HBM_PEAK_GBS},
    }
    pmc = pmc_summary()
    if pmc:
        if fp64:
            ent = pmc.get("runs", {}).get(f"{spec.N0}x{spec.N1}x{spec.N2}_fp64_resident")
            if ent:
                ff = pmc["calibration"]["fetch_factor"]
                wf = pmc["calibration"]["write_factor"]
                per_stage = 1024.0 * (ff * ent["fetch_kib"][0] + wf * ent["write_kib"][0])
                out["traffic"] = per_stage * stages
                out["hbm_counter_gbs"] = out["traffic"] / (avg_us * 1e-6) / 1e9
                out["hbm_counter_frac"] = out["hbm_counter_gbs"] / HBM_PEAK_GBS
        key = "valu_fp64" if fp64 else "valu_fp32_split"
        if key in pmc:
            out["valu_counter_flops_per_point_stage"] = pmc[key].get(
                "fp64_flops_per_point_stage" if fp64 else "fp32_flops_per_point_stage")
        if fp64 and "lds_fp64" in pmc and "lds_busy_us_per_stage" in pmc["lds_fp64"]:
            out["lds_busy_frac"] = pmc["lds_fp64"]["lds_busy_us_per_stage"] / (avg_us / stages)
    return out


def oracle_diff(u_ext, name: str):
    """max |u - u_oracle| / max |u_oracle| over the sampled stored points of the
    committed converged oracle solution `name` (tests/golden, written by the
    oracle alone), or None when the file is absent."""
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        idx, uo, umax = z["idx"], z["u"], float(z["max_abs_u"])
    return float(np.abs(np.asarray(u_ext).reshape(-1)[idx] - uo).max() / umax)


def copy_bandwidth(torch, nbytes: int = 1 << 30) -> float:
    """Device-to-device copy rate (GB/s, read + write bytes) of a plain 1 GiB copy,
    timed with events: the box's practical HBM ceiling, reported beside the
    nominal 8 TB/s."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(5):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def kernel_profile(shape_s: str, prec_s: str, variant: int = 0, coords: str = "sinhsymtp") -> int:
    """Only the stage kernels at one shape (for rocprofv3 counter passes): the
    paper-scale punctures on SinhSymTP, or on the Cartesian cube (rmax 32)."""
    import torch

    import paper_2501_14030_amd as hr
    from paper_2501_14030_amd import workloads

    shape = tuple(int(x) for x in shape_s.split("x"))
    torch.cuda.set_device(0)
    if coords == "cartesian":
        w = workloads.paper_scale_cartesian()
        g = hr.grid_create(hr.CARTESIAN, *shape, 10, params=hr.default_params(rmax=w.grid.rmax))
    else:
        w = workloads.paper_scale()
        g = hr.grid_create(0, *shape, 10, params=hr.default_params(bscale=w.grid.bscale))
    if variant:
        g.set_kernel_config(variant=variant)
    g.set_punctures(*w.punctures.as_tuple())
    prec = {"fp64": hr.FP64, "fp32": hr.FP32, "split": hr.FP32_FP64FINISH}[prec_s]
    us = g.time_stage_kernels(w.eta, w.kappa, 0.0, 3, prec)
    print(json.dumps({"shape": shape, "prec": prec_s, "avg_launch_us": list(us),
                      "config": g.kernel_config(), "kernel_sha": kernel_sha()}), flush=True)
    return 0


def copy_calibration() -> int:
    """A plain device copy of known size (1 GiB each way), for scaling the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch

    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 8}), flush=True)
    return 0


def catalog_run(n: int, precision_s: str, autotune: bool, max_steps: int,
                budget: int) -> int:
    print(json.dumps(catalog_result(n, precision_s, autotune, max_steps, budget)), flush=True)
    return 0


def catalog_result(n: int, precision_s: str, autotune: bool, max_steps: int,
                   budget: int, mlp=None) -> dict:
    """The seeded BBH catalog (q ~ U[1,10], D ~ U[6,20], |chi| ~ U[0,0.8] isotropic,
    grids drawn from 64x64x8, 128x128x16, 256x256x32) relaxed to the catalog
    tolerance of each shape (1e-10; 1e-9 at 256x256x32, whose FP64 residual
    floor is above 1e-10) by the batched path: one persistent launch per RK
    stage over every grid still relaxing in its group, graph-captured per check
    interval; groups sized to the Infinity Cache (budget bytes, 0: one group);
    eta per grid from its dt. With autotune, the batch-level tile tuner
    (catalog.autotune_batches) picks each batched composition's phi chunk on
    fresh grids before the timed region. With a trained warm-start network
    (mlp), the same grids are relaxed again from its prediction
    (catalog.warm_start_catalog: inference, the batched smoothing phase, then
    the same relaxation), timed from the inference on."""
    import torch

    import paper_2501_14030_amd as hr
    from paper_2501_14030_amd import catalog, warmstart, workloads

    torch.cuda.set_device(0)
    prec = hr.FP64 if precision_s == "fp64" else hr.FP32_FP64FINISH
    if budget <= 0:
        budget = 1 << 62
    ws = workloads.catalog(n, seed=14030)
    grids = [warmstart.make_grids([w], w.grid.shape)[0] for w in ws]
    etas = [workloads.eta_for_dt(g.suggest_dt(0.5)) for g in grids]
    tols = [workloads.catalog_tol(g.N) for g in grids]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    tuned = {}
    t_tune = 0.0
    if autotune:
        # batch-level tile tuning on fresh grids, outside the timed region
        t0 = time.perf_counter()
        tuned = catalog.autotune_batches(ws, grids, prec,
                                         catalog.plan_groups(grids, prec, budget, cus), etas,
                                         log=log)
        t_tune = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, resid = catalog.relax_catalog(grids, etas, tols, prec, max_steps=max_steps,
                                         budget=budget, log=log)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    upd = sum(g.n_interior * 4 * st for g, st in zip(grids, steps))
    conv = sum(1 for r, tol in zip(resid, tols) if r < tol)
    by_shape = {}
    for g, st in zip(grids, steps):
        k = "x".join(map(str, g.N))
        e = by_shape.setdefault(k, {"grids": 0, "tol": workloads.catalog_tol(g.N), "steps": []})
        e["grids"] += 1
        e["steps"].append(st)
    for e in by_shape.values():
        e["mean_steps"] = float(np.mean(e["steps"]))
        e["max_steps"] = int(np.max(e.pop("steps")))
    out = {"workload": f"seeded catalog of {n} BBH configurations (seed 14030: q ~ U[1,10], "
                       "D ~ U[6,20], |chi| ~ U[0,0.8] isotropic, Newtonian quasi-circular "
                       "momenta), grids drawn from SinhSymTP 64x64x8, 128x128x16, 256x256x32, "
                       "order 10, each relaxed from rest to its catalog tolerance",
           "catalog_configs": n, "precision": precision_s, "converged": conv,
           "wall_s": el, "grid_point_rhs_updates_per_s": upd / el,
           "groups": len(catalog.plan_groups(
               grids, prec, budget, torch.cuda.get_device_properties(0).multi_processor_count)),
           "cache_budget_bytes": budget,
           "by_shape": by_shape,
           "autotune_s": t_tune,
           "autotuned": {" + ".join("x".join(map(str, sh)) for sh in k):
                         {"chunk": v[0], "ms_per_40_steps": {str(c): t * 1e3 for c, t in v[1].items()}}
                         for k, v in tuned.items()}}
    if mlp is not None:
        for w, g in zip(ws, grids):
            g.set_punctures(*w.punctures.as_tuple())   # back to rest
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ns = catalog.warm_start_catalog(mlp, ws, grids, etas)
        torch.cuda.synchronize()
        t_ws = time.perf_counter() - t0
        steps_w, resid_w = catalog.relax_catalog(grids, etas, tols, prec, max_steps=max_steps,
                                                 budget=budget)
        torch.cuda.synchronize()
        el_w = time.perf_counter() - t0
        by_w = {}
        for g, st, st0 in zip(grids, steps_w, steps):
            e = by_w.setdefault("x".join(map(str, g.N)), {"steps": [], "ratio": []})
            e["steps"].append(ns + st)
            e["ratio"].append((ns + st) / st0)
        out["warm_start"] = {
            "network": "the warm-start MLP trained in this run (warmstart.RECIPE)",
            "smoothing_steps": ns,
            "converged": sum(1 for r, tol in zip(resid_w, tols) if r < tol),
            "wall_s": el_w, "inference_and_smoothing_s": t_ws,
            "speedup_vs_cold": el / el_w,
            "by_shape": {k: {"mean_steps": float(np.mean(v["steps"])),
                             "mean_steps_ratio_vs_cold": float(np.mean(v["ratio"])),
                             "max_steps_ratio_vs_cold": float(np.max(v["ratio"]))}
                         for k, v in by_w.items()}}
        log(f"catalog warm-started: {el_w:.1f} s ({el / el_w:.2f}x the cold catalog)")
    for g in grids:
        g.close()
    return out


def run_solve(hr, torch, g, w, precision, times=None):
    """One solve: sources on the device (u = v = 0), then relaxation to tol.
    With `times`, appends (sources seconds, relaxation seconds)."""
    t0 = time.perf_counter()
    g.set_punctures(*w.punctures.as_tuple())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = g.relax(w.eta, w.kappa, 0.0, w.n_steps, w.tol, check_every=w.check_every,
                  precision=precision)
    torch.cuda.synchronize()
    if times is not None:
        times.append((t1 - t0, time.perf_counter() - t1))
    return res


def timed_solves(hr, torch, g, w, precision, steps, warmup, label, timing=None):
    """Warm-up solves, then `steps` timed solves. With a dict `timing`, the
    resident launches of the timed solves are timed by the library (HIP events
    inside each dispatch) and their totals stored in it."""
    for i in range(warmup):
        r = run_solve(hr, torch, g, w, precision)
        log(f"{label} warmup {i}: status {r.status} steps {r.steps_taken} residual {r.residual:.3e}")
    if timing is not None:
        g.set_launch_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, times = [], []
    for i in range(steps):
        r = run_solve(hr, torch, g, w, precision, times)
        results.append(r)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if timing is not None:
        timing.update(g.launch_timing())
        g.set_launch_timing(False)
    for i, r in enumerate(results):
        log(f"{label} solve {i}: status {r.status} rk4 steps {r.steps_taken} "
            f"(fp32 {r.fp32_steps}) residual {r.residual:.3e} ({times[i][1] * 1e3:.2f} ms)")
        if r.status != hr.OK:
            raise RuntimeError(f"{label} solve did not converge: status {r.status}")
    return results, t1 - t0, times


def precision_form_runs(hr, torch):
    """The single-precision forms on the 8th-order precision-form grids
    (equal-mass small-case physics), each relaxed once to residual 1e-10: FP64,
    the split FP32 bulk with an FP64 finish, and the same with bfloat16 metric
    factors; errors are stated against the FP64 solution of the same grid."""
    from paper_2501_14030_amd import workloads
    res = {}
    for shape in ((128, 128, 16), (256, 256, 32)):
        w = workloads.precision_form(*shape)
        s = w.grid
        g = hr.grid_create(s.coords, s.N0, s.N1, s.N2, s.fd_order,
                           params=hr.default_params(bscale=s.bscale))
        g.set_fp32_switch(0.0, 8, 0)
        entry = {"grid": list(shape), "fd_order": s.fd_order, "eta": w.eta, "tol": w.tol}
        u64 = None
        for label, prec, bits in (("fp64", hr.FP64, 32), ("split", hr.FP32_FP64FINISH, 32),
                                  ("split_bf16_factors", hr.FP32_FP64FINISH, 16)):
            g.set_factor_storage(bits)
            times = []
            r = run_solve(hr, torch, g, w, prec, times)
            u = g.get_u()
            if u64 is None:
                u64 = u
            e = {"time_to_residual_s": times[0][1], "rk4_steps_to_tol": r.steps_taken,
                 "fp32_steps": r.fp32_steps, "final_residual": r.residual, "status": r.status,
                 "updates_per_s": s.n_interior * 4 * r.steps_taken / times[0][1],
                 "max_rel_diff_u_vs_fp64": float(np.abs(u - u64).max() / np.abs(u64).max()),
                 "max_rel_diff_u_vs_oracle": oracle_diff(
                     g.get_u(extended=True), f"precision_form_{shape[0]}x{shape[1]}x{shape[2]}")}
            log(f"precision form {s.name()} {label}: {r.steps_taken} steps ({r.fp32_steps} fp32), "
                f"residual {r.residual:.3e}, {times[0][1]:.3f} s, "
                f"diff vs fp64 {e['max_rel_diff_u_vs_fp64']:.2e}")
            entry[label] = e
        entry["oracle_reference"] = (f"converged FP64 oracle solution at 4096 seeded stored "
                                     f"points and the largest |u| (tests/golden/oracle_"
                                     f"precision_form_{shape[0]}x{shape[1]}x{shape[2]}.npz)")
        res[s.name()] = entry
        g.close()
    return res


def multi_patch_runs(hr, torch, w, u_ref, n_max: int = 7):
    """The independent-patches experiment of Sec. 4 (multiple, independent
    patches): N = 1 .. n_max identical paper-scale grids relaxed from u = v = 0
    to the tolerance, (a) as one batch (one persistent launch per RK stage over
    every grid, graph-captured per check interval) and (b) one after another
    with the single-grid path. t_N counts the sources and the relaxation, after
    one untimed run of the same N; t_N / t_1 is the quantity of the paper's
    figure (it found the GPU code close to linear in N)."""
    s = w.grid
    prm = hr.default_params(amax=s.amax, sinhwaa=s.sinhwaa, bscale=s.bscale, rmax=s.rmax)
    grids = [hr.grid_create(s.coords, s.N0, s.N1, s.N2, s.fd_order, params=prm)
             for _ in range(n_max)]
    for g in grids:
        run_solve(hr, torch, g, w, hr.FP64)   # untimed: workspace bound, graphs captured
    rows = []
    for n in range(1, n_max + 1):
        sub = grids[:n]
        b = hr.Batch(sub)
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for g in sub:
                g.set_punctures(*w.punctures.as_tuple())
            torch.cuda.synchronize()
            res = b.relax([w.eta] * n, w.kappa, n_steps=w.n_steps, tol=w.tol,
                          check_every=w.check_every)
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
        b.close()
        steps_b = [r.steps_taken for r in res]
        if any(r.status != hr.OK for r in res):
            raise RuntimeError(f"multi-patch batch of {n} did not converge")
        diff = max(float(np.abs(g.get_u() - u_ref).max() / np.abs(u_ref).max()) for g in sub)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq = [run_solve(hr, torch, g, w, hr.FP64) for g in sub]
        torch.cuda.synchronize()
        tq = time.perf_counter() - t0
        if any(r.status != hr.OK for r in seq):
            raise RuntimeError(f"multi-patch sequential run of {n} did not converge")
        rows.append({"n": n, "batched_s": tb, "sequential_s": tq, "rk4_steps_batched": steps_b,
                     "rk4_steps_sequential": [r.steps_taken for r in seq],
                     "max_rel_diff_u_batched_vs_single": diff})
        log(f"multi-patch N={n}: batched {tb:.3f} s (steps {steps_b[0]}), sequential {tq:.3f} s, "
            f"batched u vs single solve {diff:.2e}")
    for g in grids:
        g.close()
    t1b, t1q = rows[0]["batched_s"], rows[0]["sequential_s"]
    best1 = min(t1b, t1q)
    for r in rows:
        r["batched_over_t1"] = r["batched_s"] / t1b
        r["sequential_over_t1"] = r["sequential_s"] / t1q
        r["best_over_best_t1"] = min(r["batched_s"], r["sequential_s"]) / best1
    return {"workload": f"N identical {s.name()} relaxations from u = v = 0 to residual "
                        f"{w.tol} (paper-scale punctures, eta {w.eta}), N = 1..{n_max}",
            "rows": rows}


def cartesian_runs(hr, torch, steps: int, warmup: int):
    """The paper-scale punctures on the Cartesian cube 128^3 ([-32, 32]^3, 10th
    order, eta 0.03; the Cartesian-like family): FP64 solves to residual 1e-10
    on the z-column stage kernel (face points in the same launch), its
    per-stage times with the HBM roofline of their algorithmic bytes, the
    split-state form's solves, and the errors against the committed converged
    oracle solution."""
    from paper_2501_14030_amd import workloads

    w = workloads.paper_scale_cartesian()
    s = w.grid
    g = hr.grid_create(s.coords, s.N0, s.N1, s.N2, s.fd_order,
                       params=hr.default_params(rmax=s.rmax))
    rs, ts, tms = timed_solves(hr, torch, g, w, hr.FP64, steps, warmup, "cartesian fp64")
    u64 = g.get_u(extended=True)
    diff = oracle_diff(u64, "paper_scale_cartesian_128")
    # the split-state form (FP32 increment on the FP64 base, FP64 finish)
    g.set_fp32_switch(0.0, 8, 0)
    rs32, ts32, _ = timed_solves(hr, torch, g, w, hr.FP32_FP64FINISH, steps, warmup,
                                 "cartesian split")
    u32 = g.get_u(extended=True)
    diff32 = oracle_diff(u32, "paper_scale_cartesian_128")
    us = g.time_stage_kernels(w.eta, w.kappa, 0.0, 5, hr.FP64)
    byts = stage_algorithmic_bytes(s, 8, cart=True)
    agg = sum(byts) / (sum(us[:4]) * 1e-6) / 1e9
    tr = measured_traffic(s.shape, "fp64", cart=True)
    out = {
        "workload": f"paper-scale punctures on the Cartesian cube {s.N0}^3, [-{s.rmax:g}, "
                    f"{s.rmax:g}]^3, 10th-order FD, eta {w.eta}, to residual 1e-10",
        "value": sum(s.n_interior * 4 * r.steps_taken for r in rs) / ts,
        "unit": "grid-pt RHS updates/s",
        "time_to_residual_s": ts / steps,
        "relax_median_s": float(np.median([t[1] for t in tms])),
        "rk4_steps_to_tol": rs[-1].steps_taken,
        "final_residual": rs[-1].residual,
        "max_rel_diff_u_vs_oracle": diff,
        "oracle_reference": "converged FP64 oracle solution at 4096 seeded evolved points and "
                            "the largest |u| (tests/golden/oracle_paper_scale_cartesian_128.npz)",
        "mixed": {"precision": "split state: FP32 increment on the FP64 base, FP64 finish",
                  "time_to_residual_s": ts32 / steps,
                  "speedup_vs_fp64": ts / ts32,
                  "rk4_steps_to_tol": rs32[-1].steps_taken, "fp32_steps": rs32[-1].fp32_steps,
                  "final_residual": rs32[-1].residual,
                  "max_rel_diff_u_vs_fp64": float(np.abs(u32 - u64).max() / np.abs(u64).max()),
                  "max_rel_diff_u_vs_oracle": diff32},
        "roofline": {"bound": "hbm", "achieved": agg, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": agg / HBM_PEAK_GBS, "traffic": tr,
                     "traffic_over_algorithmic": (tr / (sum(byts) / 4)) if tr else None,
                     "kernel": "Cartesian z-column kernel (8 planes per block) with its "
                               "face-point blocks, one launch per stage (FP64, order 10), "
                               "mean over stages 1-4",
                     "kernel_config": g.resolved_kernel(hr.FP64),
                     "avg_stage_us": [float(x) for x in us[:4]],
                     "algorithmic_bytes_per_stage": byts},
    }
    log(f"cartesian: {rs[-1].steps_taken} steps, {ts / steps * 1e3:.1f} ms, "
        f"{out['value'] / 1e9:.1f} G updates/s, {agg / 1e3:.2f} TB/s, vs oracle {diff}; "
        f"split {ts32 / steps * 1e3:.1f} ms")
    g.close()
    return out


def warm_start_runs(hr, torch, g, w, steps, steps_cold, t_cold, u_cold, sols=None, keep=None):
    """The learned warm start. An MLP trained inside this run (warmstart.RECIPE:
    4096 catalog solves at 64x64x8, 2048 sampled points each) predicts u; the
    warm start is that prediction, 100 RK4 steps at ten times the damping
    (which remove its small-scale error) and v = eta u, then the relaxation to
    the same tolerance. Reported on the paper-scale configuration (timed solves
    include inference and smoothing; data generation and training are reported
    separately) with the control (from rest through the same smoothing phase),
    and on 64 held-out catalog configurations at 128x128x16 (seed 14032), the
    distribution the network is trained on."""
    from paper_2501_14030_amd import warmstart, workloads
    from paper_2501_14030_amd.mlp import config_features

    mlp, info = warmstart.fit(log=lambda m: None)
    log(f"warm start: {info['train_configs']} training solves in {info['data_s']:.1f} s, "
        f"{info['samples']} samples trained in {info['train_s']:.1f} s "
        f"(loss {info['final_loss']:.3e})")
    # q = 1, chi1 = chi2 = (0, 0, 0.8) (S = 0.2 on m = 0.5), |P| = 0.095, D = 10
    # (1.2 times the Newtonian quasi-circular momentum, inside the training spread)
    cfg = config_features(1.0, [0.0, 0.0, 0.8], [0.0, 0.0, 0.8], 0.095, 10.0)
    m, ns = warmstart.SMOOTH
    out = dict(info)
    out["smoothing"] = {"damping_multiple": m, "steps": ns}
    for label, prec in (("fp64", hr.FP64), ("split", hr.FP32_FP64FINISH), ("control", hr.FP64)):
        times, res = [], None
        for _ in range(steps):
            g.set_punctures(*w.punctures.as_tuple())
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if label == "control":   # from rest through the same smoothing phase
                g.relax(m * w.eta, w.kappa, 0.0, ns, 0.0, check_every=ns)
                g.reset_v(w.eta)
                done = ns
            else:
                done = warmstart.warm_start(mlp, g, cfg, w.eta)
            res = g.relax(w.eta, w.kappa, 0.0, w.n_steps, w.tol, check_every=w.check_every,
                          precision=prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            if res.status != hr.OK:
                raise RuntimeError(f"warm-started {label} solve did not converge")
        u = g.get_u()
        if sols is not None and label != "control":
            sols[f"warm_{label}"] = g.get_u(extended=True)
        out[label] = {"time_to_residual_s": float(np.median(times)),
                      "rk4_steps_to_tol": done + res.steps_taken, "fp32_steps": res.fp32_steps,
                      "final_residual": res.residual,
                      "max_rel_diff_u_vs_cold_fp64": float(np.abs(u - u_cold).max() /
                                                           np.abs(u_cold).max())}
        log(f"warm start {label}: {done + res.steps_taken} steps, "
            f"{np.median(times) * 1e3:.2f} ms")
    out["fp64"]["steps_vs_cold"] = out["fp64"]["rk4_steps_to_tol"] / steps_cold
    out["fp64"]["speedup_vs_cold_fp64"] = t_cold / out["fp64"]["time_to_residual_s"]
    out["split"]["speedup_vs_cold_fp64"] = t_cold / out["split"]["time_to_residual_s"]
    test_ws = workloads.catalog(64, seed=14032, shapes=((128, 128, 16),))
    ev = warmstart.evaluate(mlp, test_ws, (128, 128, 16), tol=1e-10, batch=32,
                            log=lambda m: None)
    cold = np.array(ev["cold_steps"])
    warm = np.array(ev["warm_steps"])
    ctl = np.array(ev["cold_smooth_steps"])
    out["held_out"] = {
        "workload": "64 held-out catalog configurations (seed 14032) at SinhSymTP 128x128x16, "
                    "order 10, relaxed to 1e-10 in batches of 32 each way",
        "mean_steps_cold": float(cold.mean()), "mean_steps_warm": float(warm.mean()),
        "mean_steps_control": float(ctl.mean()),
        "frac_configs_fewer_steps_than_cold": float(np.mean(warm < cold)),
        "steps_ratio_min_max": [float((warm / cold).min()), float((warm / cold).max())],
        "mean_steps_ratio_warm_vs_cold": float(warm.mean() / cold.mean()),
        "mean_steps_ratio_warm_vs_control": float(warm.mean() / ctl.mean()),
        "time_cold_s": ev["cold_s"], "time_warm_s": ev["warm_s"],
        "time_control_s": ev["cold_smooth_s"],
        "prediction_median_rel_err": float(np.median(ev["pred_rel_err"])),
        "prediction_median_rel_err_p90": float(np.percentile(ev["pred_rel_err"], 90)),
    }
    log(f"warm start held out: steps {warm.mean():.0f} vs cold {cold.mean():.0f} "
        f"(control {ctl.mean():.0f}), time {ev['warm_s']:.3f} vs {ev['cold_s']:.3f} s")
    if keep is not None:   # the caller warm-starts the catalog with it, then closes it
        keep.append(mlp)
    else:
        mlp.close()
    return out


def cpu_baseline(w, budget_s: float, full_s: float, steps_gpu: int):
    """The oracle as it is, on the host cores. When the whole solve to the
    tolerance fits in `full_s` seconds (estimated from two steps) it runs the
    whole solve, exactly as the GPU does (residual every check_every steps);
    else a bounded sample of RK4 steps of the same grid from the same initial
    state. Returns the entry and the oracle's final u (extended layout) when
    the whole solve ran, else None."""
    import oracle

    oracle.build()
    spec = w.grid
    og = oracle.OracleGrid(spec.coords, spec.N0, spec.N1, spec.N2, spec.fd_order,
                           amax=spec.amax, sinhwaa=spec.sinhwaa, bscale=spec.bscale,
                           rmax=spec.rmax)
    og.set_punctures(*w.punctures.as_tuple())
    dt = og.suggest_dt(w.cfl)
    t0 = time.perf_counter()
    og.rk4_steps(w.eta, w.kappa, dt, 2)
    per_step = (time.perf_counter() - t0) / 2
    u_full = None
    if per_step * steps_gpu <= full_s:
        og.set_punctures(*w.punctures.as_tuple())
        t0 = time.perf_counter()
        st, n, hist = og.relax(w.eta, w.kappa, dt, w.n_steps, w.tol, w.check_every)
        el = time.perf_counter() - t0
        u, _ = og.state()
        ng = og.NG
        u_full = u[ng:ng + spec.N2, ng:ng + spec.N1, ng:ng + spec.N0 + ng]
        sample = (f"the whole solve: {n} RK4 steps of {spec.name()} from rest to residual "
                  f"{hist[-1]:.3e} (status {st}), residual every {w.check_every} steps ({el:.1f} s)")
    else:
        n = max(2, int(budget_s / max(per_step, 1e-6)))
        t0 = time.perf_counter()
        og.rk4_steps(w.eta, w.kappa, dt, n)
        el = time.perf_counter() - t0
        sample = (f"{n} RK4 steps of {spec.name()} from rest ({el:.1f} s); time to residual "
                  f"1e-10 extrapolates as steps_to_tol / {n / el:.2f} steps/s")
    upd = spec.n_interior * 4 * n / el
    cores = oracle.num_threads()
    # the same on one thread (fewer steps: about a third of the budget)
    oracle.set_num_threads(1)
    n1 = max(1, int(budget_s / 3 / max(per_step * cores, 1e-6)))
    t0 = time.perf_counter()
    og.rk4_steps(w.eta, w.kappa, dt, n1)
    el1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    return {"value": upd, "unit": "grid-pt RHS updates/s", "cores": cores,
            "kind": "oracle", "sample": sample, "oracle_steps": n,
            "value_1_thread": spec.n_interior * 4 * n1 / el1,
            "sample_1_thread": f"{n1} RK4 steps, same grid, 1 thread ({el1:.1f} s)"}, u_full


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-full-seconds", type=float, default=40.0,
                    help="run the oracle's whole solve when it is estimated to fit in this time")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-spherical", action="store_true")
    ap.add_argument("--no-precision-form", action="store_true")
    ap.add_argument("--no-cartesian", action="store_true")
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--no-multi-patch", action="store_true")
    ap.add_argument("--no-catalog", action="store_true",
                    help="skip the 64-configuration catalog (FP32 + FP64 finish) entry")
    ap.add_argument("--kernel-profile", metavar="N0xN1xN2", default=None,
                    help="only run the stage kernels at this shape (counter passes)")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "split"])
    ap.add_argument("--coords", default="sinhsymtp", choices=["sinhsymtp", "cartesian"],
                    help="grid family of --kernel-profile")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--catalog", type=int, default=0, metavar="N",
                    help="relax the seeded N-configuration catalog with the batched path")
    ap.add_argument("--catalog-prec", default="fp64", choices=["fp64", "split"])
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the default bench's catalog without batch tile tuning")
    ap.add_argument("--cache-budget", type=int, default=200 << 20,
                    help="catalog: per-stage working set of one batch (bytes; 0 = one batch)")
    ap.add_argument("--max-steps", type=int, default=60000)
    ap.add_argument("--variant", type=int, default=0,
                    help="stage kernel variant (0 automatic, 1 plane, 2 columns, 3 resident)")
    args = ap.parse_args()
    if args.catalog:
        return catalog_run(args.catalog, args.catalog_prec, args.autotune, args.max_steps,
                           args.cache_budget)
    if args.kernel_profile:
        return kernel_profile(args.kernel_profile, args.prec, args.variant, args.coords)
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the relaxation of "
              "one grid runs on a single GPU and is not sharded across GPUs.", file=sys.stderr)
        return 2

    import torch

    import paper_2501_14030_amd as hr
    from paper_2501_14030_amd import workloads

    hr.load_library()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    w = workloads.paper_scale(workloads.SINHSYMTP, 10)
    spec = w.grid
    log(f"workload {w.label}: eta {w.eta} cfl {w.cfl} tol {w.tol} check every {w.check_every}")
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    g = hr.grid_create(spec.coords, spec.N0, spec.N1, spec.N2, spec.fd_order,
                       params=hr.default_params(amax=spec.amax, sinhwaa=spec.sinhwaa,
                                                bscale=spec.bscale, rmax=spec.rmax))
    g.set_punctures(*w.punctures.as_tuple())
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup   # host tables, device workspace, sources
    if args.variant:
        g.set_kernel_config(variant=args.variant)
    tim64, tim32 = {}, {}
    res64, t64, tm64 = timed_solves(hr, torch, g, w, hr.FP64, args.steps, args.warmup, "fp64",
                                    tim64)
    steps64 = res64[-1].steps_taken
    upd64 = sum(spec.n_interior * 4 * r.steps_taken for r in res64) / t64
    u64 = g.get_u()
    sols = {"fp64": g.get_u(extended=True)}   # compared with the oracle's solve below
    out = {
        "metric": METRIC,
        "value": upd64,
        "unit": "grid-pt RHS updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t64 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "paper-scale single solve: SinhSymTP 128x128x16, 10th-order FD, "
                        "q=1 punctures at z=+-5, |P|=0.095 along +-y, S=(0,0,0.2), relax from "
                        "u=v=0 to residual L2 < 1e-10 (one step = one whole solve)",
            "grid": list(spec.shape), "fd_order": spec.fd_order, "eta": w.eta, "cfl": w.cfl,
            "tol": w.tol, "check_every": w.check_every,
        },
        "time_to_residual_s": t64 / args.steps,
        "time_to_residual": {
            "relax_median_s": float(np.median([t[1] for t in tm64])),
            "relax_per_solve_s": [t[1] for t in tm64],
            "sources_median_s": float(np.median([t[0] for t in tm64])),
            "first_setup_s": setup_s,
            "note": "relax = setup excluded; + sources = the timed step; first_setup = grid "
                    "creation, host tables, workspace allocation and binding, sources (once)",
        },
        "rk4_steps_to_tol": steps64,
        "final_residual": res64[-1].residual,
        "kernel": g.resolved_kernel(hr.FP64),
    }
    if not args.no_mixed:
        g.set_fp32_switch(0.0, 8, 0)  # FP64 finish below 10 x tol
        res32, t32, tm32 = timed_solves(hr, torch, g, w, hr.FP32_FP64FINISH, args.steps, 0,
                                        "fp32+fp64", tim32)
        u32 = g.get_u()
        sols["mixed"] = g.get_u(extended=True)
        out["mixed"] = {
            "precision": "FP32 bulk (split state: FP64 base + FP32 increment, FP64 slopes, "
                         "rebase and residual every check) + plain FP64 finish below 10 x tol",
            "value": sum(spec.n_interior * 4 * r.steps_taken for r in res32) / t32,
            "time_to_residual_s": t32 / args.steps,
            "relax_median_s": float(np.median([t[1] for t in tm32])),
            "rk4_steps_to_tol": res32[-1].steps_taken,
            "fp32_steps": res32[-1].fp32_steps,
            "final_residual": res32[-1].residual,
            "max_rel_diff_u_vs_fp64": float(np.abs(u32 - u64).max() / np.abs(u64).max()),
            "speedup_time_to_residual": (t64 / args.steps) / (t32 / args.steps),
        }
        # fixed form: single precision for 95% of the FP64 form's steps to the
        # tolerance (at check granularity), then FP64 to the tolerance
        cap = int(round(0.95 * steps64 / w.check_every)) * w.check_every
        g.set_fp32_switch(1e-300, 1 << 30, cap)
        resf, tf, tmf = timed_solves(hr, torch, g, w, hr.FP32_FP64FINISH, args.steps, 0,
                                     "fp32 95% fixed")
        uf = g.get_u()
        sols["mixed_fixed_95"] = g.get_u(extended=True)
        out["mixed"]["fixed_95"] = {
            "time_to_residual_s": tf / args.steps,
            "relax_median_s": float(np.median([t[1] for t in tmf])),
            "rk4_steps_to_tol": resf[-1].steps_taken,
            "fp32_steps": resf[-1].fp32_steps,
            "final_residual": resf[-1].residual,
            "max_rel_diff_u_vs_fp64": float(np.abs(uf - u64).max() / np.abs(u64).max()),
        }
        g.set_fp32_switch(0.0, 8, 0)
    nets = []   # the warm-start network, kept for the catalog entry
    if not args.no_warm_start:
        out["warm_start"] = warm_start_runs(hr, torch, g, w, args.steps, steps64,
                                            float(np.median([t[1] for t in tm64])), u64, sols,
                                            keep=nets)
    if not args.no_spherical:
        # the same physics on the Spherical 128x64x8 grid (rmax 100), its own eta
        ws = workloads.paper_scale(workloads.SPHERICAL, 10)
        ss = ws.grid
        gs = hr.grid_create(ss.coords, ss.N0, ss.N1, ss.N2, ss.fd_order,
                            params=hr.default_params(rmax=ss.rmax))
        rs64, ts64, tms64 = timed_solves(hr, torch, gs, ws, hr.FP64, args.steps, args.warmup,
                                         "spherical fp64")
        us64 = gs.get_u()
        ds64 = oracle_diff(gs.get_u(extended=True), "paper_scale_spherical_128x64x8")
        gs.set_fp32_switch(0.0, 8, 0)
        rs32, ts32, tms32 = timed_solves(hr, torch, gs, ws, hr.FP32_FP64FINISH, args.steps, 0,
                                         "spherical fp32+fp64")
        us32 = gs.get_u()
        ds32 = oracle_diff(gs.get_u(extended=True), "paper_scale_spherical_128x64x8")
        out["spherical"] = {
            "workload": f"paper-scale Spherical {ss.N0}x{ss.N1}x{ss.N2}, 10th-order FD, "
                        f"rmax {ss.rmax}, same punctures, eta {ws.eta}, to residual 1e-10",
            "value": sum(ss.n_interior * 4 * r.steps_taken for r in rs64) / ts64,
            "time_to_residual_s": ts64 / args.steps,
            "relax_median_s": float(np.median([t[1] for t in tms64])),
            "rk4_steps_to_tol": rs64[-1].steps_taken,
            "final_residual": rs64[-1].residual,
            "kernel": gs.resolved_kernel(hr.FP64),
            "mixed_value": sum(ss.n_interior * 4 * r.steps_taken for r in rs32) / ts32,
            "mixed_time_to_residual_s": ts32 / args.steps,
            "mixed_rk4_steps_to_tol": rs32[-1].steps_taken,
            "mixed_fp32_steps": rs32[-1].fp32_steps,
            "mixed_max_rel_diff_u_vs_fp64": float(np.abs(us32 - us64).max() / np.abs(us64).max()),
            "max_rel_diff_u_vs_oracle": ds64,
            "mixed_max_rel_diff_u_vs_oracle": ds32,
            "oracle_reference": "converged FP64 oracle solution at 4096 seeded stored points and "
                                "the largest |u| "
                                "(tests/golden/oracle_paper_scale_spherical_128x64x8.npz)",
        }
        gs.close()
    if not args.no_cartesian:
        out["cartesian"] = cartesian_runs(hr, torch, args.steps, 1)
    if not args.no_precision_form:
        out["precision_form"] = precision_form_runs(hr, torch)
    if not args.no_multi_patch:
        out["multi_patch"] = multi_patch_runs(hr, torch, w, u64)
    if not args.no_catalog:
        log("catalog: 64 configurations, FP32 + FP64 finish ...")
        out["catalog"] = catalog_result(64, "split", not args.no_autotune, args.max_steps,
                                        args.cache_budget, nets[0] if nets else None)
        log(f"catalog: {out['catalog']['wall_s']:.1f} s, "
            f"{out['catalog']['grid_point_rhs_updates_per_s'] / 1e9:.1f} G updates/s")
    for net in nets:
        net.close()
    # roofline of the dominant kernel: the resident RK4 kernel at this size,
    # timed on the launches of the timed solves themselves
    g.set_punctures(*w.punctures.as_tuple())
    copy = copy_bandwidth(torch)
    if g.resolved_kernel(hr.FP64)["variant"] == 3 and tim64.get("launches"):
        out["roofline"] = resident_roofline(hr, spec, hr.FP64, tim64)
    else:
        out["roofline"] = roofline_entry(g, hr, spec, w, hr.FP64)
    if tim32.get("launches"):
        out["roofline_split"] = resident_roofline(hr, spec, hr.FP32_FP64FINISH, tim32)
    out["roofline_fp32"] = roofline_entry(g, hr, spec, w, hr.FP32)
    for k in ("roofline", "roofline_fp32", "roofline_split"):
        if k in out and out[k]["unit"] == "GB/s":
            out[k]["copy_gbs"] = copy
            out[k]["frac_of_copy"] = out[k]["achieved"] / copy
    out["copy_gbs"] = copy
    if not args.no_large:
        # the paper's roofline grid, 512x512x64: working set well beyond the caches
        big = workloads.GridSpec(0, 512, 512, 64, 10, bscale=spec.bscale)
        gb = hr.grid_create(0, 512, 512, 64, 10, params=hr.default_params(bscale=spec.bscale))
        gb.set_punctures(*w.punctures.as_tuple())
        out["roofline_512x512x64"] = roofline_entry(gb, hr, big, w, hr.FP64, nsteps=5)
        out["roofline_512x512x64_fp32"] = roofline_entry(gb, hr, big, w, hr.FP32, nsteps=5)
        gb.close()
        del gb
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb, u_or = cpu_baseline(w, args.cpu_seconds, args.cpu_full_seconds, steps64)
        cb["time_to_residual_s_extrapolated"] = steps64 * spec.n_interior * 4 / cb["value"]
        out["cpu_baseline"] = cb
        if u_or is not None:
            # every form of the paper-scale solve against the oracle's own solve
            scale = float(np.abs(u_or).max())
            errs = {k: float(np.abs(v - u_or).max() / scale) for k, v in sols.items()}
            out["max_rel_diff_u_vs_oracle"] = errs["fp64"]
            out["oracle_steps_to_tol"] = cb["oracle_steps"]
            for k, e in errs.items():
                if k == "mixed" and "mixed" in out:
                    out["mixed"]["max_rel_diff_u_vs_oracle"] = e
                elif k == "mixed_fixed_95" and "mixed" in out:
                    out["mixed"]["fixed_95"]["max_rel_diff_u_vs_oracle"] = e
                elif k.startswith("warm_") and "warm_start" in out:
                    out["warm_start"][k[5:]]["max_rel_diff_u_vs_oracle"] = e
        if "multi_patch" in out:
            # the oracle relaxes one grid after another: N times its one-grid time
            for r in out["multi_patch"]["rows"]:
                r["speedup_vs_oracle"] = (r["n"] * cb["time_to_residual_s_extrapolated"]
                                          / min(r["batched_s"], r["sequential_s"]))
    print(json.dumps(out), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
