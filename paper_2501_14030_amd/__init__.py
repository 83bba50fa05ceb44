"""MI355X hyperbolic-relaxation solver for binary-black-hole puncture data.

Thin ctypes binding over the C ABI declared in ``include/hrelax.h``; every
step of the relaxation runs in the HIP kernels of ``libhrelax.so``. PyTorch
only provides the device workspace and the HIP stream. The module-level
functions carry the ABI's names (``grid_create``, ``set_punctures``,
``relax``, ``get_u``, ``residual_l2``, ...).

The library must be built (``python -m paper_2501_14030_amd.build``); there is
no fallback implementation, and loading fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhrelax.so")

SINHSYMTP = 0
SPHERICAL = 1
SINHSPHERICAL = 2
SINHCYLINDRICAL = 3
CARTESIAN = 4            # the cube [-rmax, rmax]^3, outer layers beyond all six faces

FP64 = 0
FP32 = 1
FP32_FP64FINISH = 2

NORM_POINTS = 0
NORM_VOLUME = 1

OK = 0
EINVAL = -1
ENOMEM = -2
EDEVICE = -3
ENOTCONV = -4
ENONFINITE = -5
ESTATE = -6

_STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
                 ENOTCONV: "ENOTCONV", ENONFINITE: "ENONFINITE", ESTATE: "ESTATE"}


class HRError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GridParams(ctypes.Structure):
    _fields_ = [("amax", ctypes.c_double), ("sinhwaa", ctypes.c_double),
                ("bscale", ctypes.c_double), ("rmax", ctypes.c_double),
                ("cfl", ctypes.c_double)]


class KernelConfig(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("streaming", ctypes.c_int), ("chunk", ctypes.c_int),
                ("graph", ctypes.c_int)]


class RelaxReport(ctypes.Structure):
    _fields_ = [("steps_taken", ctypes.c_long), ("fp32_steps", ctypes.c_long),
                ("residual", ctypes.c_double), ("dt_used", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_long),
                ("n_history", ctypes.c_long), ("resident_fallbacks", ctypes.c_long)]


_dp = ctypes.POINTER(ctypes.c_double)
_lib = None

# Every symbol the header declares, with (restype, argtypes).
_SIGNATURES = {
    "hr_default_params": (None, [ctypes.POINTER(GridParams)]),
    "hr_grid_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(GridParams),
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "hr_grid_destroy": (None, [ctypes.c_void_p]),
    "hr_grid_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "hr_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "hr_grid_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p]),
    "hr_set_punctures": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp]),
    "hr_relax": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_long, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, ctypes.POINTER(RelaxReport)]),
    "hr_relax_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_long, ctypes.c_double,
                                        ctypes.c_int, ctypes.POINTER(RelaxReport)]),
    "hr_set_fp32_switch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_long]),
    "hr_reset_v": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "hr_get_u": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t]),
    "hr_get_v": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t]),
    "hr_set_u": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t]),
    "hr_set_v": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_size_t]),
    "hr_residual_l2": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "hr_suggest_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, _dp]),
    "hr_time_stage_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_long, ctypes.c_int, _dp]),
    "hr_set_kernel_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelConfig)]),
    "hr_get_kernel_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelConfig)]),
    "hr_resolved_kernel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                          ctypes.POINTER(KernelConfig)]),
    "hr_set_wait_limit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint]),
    "hr_set_launch_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hr_get_launch_timing": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.POINTER(ctypes.c_long),
                                            ctypes.POINTER(ctypes.c_long)]),
    "hr_set_outer_bc_order": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hr_set_factor_storage": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hr_set_residual_norm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]),
    "hr_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(KernelConfig), _dp]),
    "hr_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "hr_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "hr_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]),
    "hr_batch_relax": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, ctypes.c_long, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "hr_batch_destroy": (None, [ctypes.c_void_p]),
    "hr_last_error": (ctypes.c_char_p, []),
}


def _hip_runtimes_mapped() -> list:
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def load_library(path: str = LIB_PATH):
    """Loads ``libhrelax.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library {path} is missing: build it with "
            "`python -m paper_2501_14030_amd.build` (there is no fallback path)")
    # torch owns the device memory and streams; its HIP runtime must be the one
    # the library binds to, so it is loaded first (same SONAME, so the library's
    # dependency resolves to the copy already in the process).
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise RuntimeError(f"more than one HIP runtime is loaded in this process: {runtimes}")
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int, where: str) -> int:
    if status != OK:
        raise HRError(status, where, load_library().hr_last_error().decode())
    return status


def default_params(**overrides) -> GridParams:
    p = GridParams()
    load_library().hr_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, float(v))
    return p


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class RelaxResult:
    status: int
    steps_taken: int
    fp32_steps: int
    residual: float
    dt: float
    history: np.ndarray
    resident_fallbacks: int = 0


class Grid:
    """A relaxation grid bound to torch-owned device memory and a HIP stream."""

    def __init__(self, coords: int, N0: int, N1: int, N2: int, fd_order: int,
                 params: GridParams | None = None, device=None, stream=None):
        import torch  # device memory and streams only

        L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the relaxation runs only on the HIP device")
        h = ctypes.c_void_p()
        pp = ctypes.byref(params) if params is not None else None
        _check(L.hr_grid_create(int(coords), N0, N1, N2, fd_order, pp, ctypes.byref(h)),
               "hr_grid_create")
        self._h = h
        self.coords = coords
        self.N = (N0, N1, N2)
        self.fd_order = fd_order
        self.NG = fd_order // 2
        nint = ctypes.c_size_t()
        next_ = ctypes.c_size_t()
        _check(L.hr_grid_sizes(h, ctypes.byref(nint), ctypes.byref(next_)), "hr_grid_sizes")
        self.n_interior = nint.value
        self.n_extended = next_.value
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = L.hr_workspace_bytes(h)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self._ws.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        with torch.cuda.device(self.device):
            _check(L.hr_grid_bind(h, ctypes.c_void_p(aligned), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream)), "hr_grid_bind")

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hr_grid_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_punctures(self, m, x, P, S) -> None:
        m = _f64(m)
        n = len(m)
        x = _f64(x).reshape(n, 3)
        P = _f64(P).reshape(n, 3)
        S = _f64(S).reshape(n, 3)
        _check(load_library().hr_set_punctures(self._h, n, m.ctypes.data_as(_dp),
                                               x.ctypes.data_as(_dp), P.ctypes.data_as(_dp),
                                               S.ctypes.data_as(_dp)), "hr_set_punctures")

    def relax(self, eta: float, c: float = 1.0, dt: float = 0.0, n_steps: int = 1000,
              tol: float = 0.0, check_every: int = 100, precision: int = FP64,
              raise_on_error: bool = True) -> RelaxResult:
        cap = max(1, int(n_steps) // max(1, int(check_every)) + 2)
        hist = np.zeros(cap)
        rep = RelaxReport()
        rep.history = hist.ctypes.data_as(_dp)
        rep.history_cap = cap
        st = load_library().hr_relax(self._h, float(eta), float(c), float(dt), int(n_steps),
                                     float(tol), int(check_every), int(precision),
                                     ctypes.byref(rep))
        if st not in (OK, ENOTCONV, ENONFINITE) or (raise_on_error and st == ENONFINITE):
            _check(st, "hr_relax")
        return RelaxResult(st, rep.steps_taken, rep.fp32_steps, rep.residual, rep.dt_used,
                           hist[:min(rep.n_history, cap)].copy(), rep.resident_fallbacks)

    def relax_noalloc(self, eta: float, c: float = 1.0, dt: float = 0.0, n_steps: int = 1000,
                      tol: float = 0.0, check_every: int = 100,
                      raise_on_error: bool = True) -> RelaxResult:
        """hr_relax_noalloc: the FP64 relaxation with the library's static
        device scratch in place of the workspace's (allocates nothing)."""
        cap = max(1, int(n_steps) // max(1, int(check_every)) + 2)
        hist = np.zeros(cap)
        rep = RelaxReport()
        rep.history = hist.ctypes.data_as(_dp)
        rep.history_cap = cap
        st = load_library().hr_relax_noalloc(self._h, float(eta), float(c), float(dt),
                                             int(n_steps), float(tol), int(check_every),
                                             ctypes.byref(rep))
        if st not in (OK, ENOTCONV, ENONFINITE) or (raise_on_error and st == ENONFINITE):
            _check(st, "hr_relax_noalloc")
        return RelaxResult(st, rep.steps_taken, rep.fp32_steps, rep.residual, rep.dt_used,
                           hist[:min(rep.n_history, cap)].copy(), rep.resident_fallbacks)

    def set_fp32_switch(self, switch_residual: float = 0.0, stall_checks: int = 8,
                        max_fp32_steps: int = 0) -> None:
        _check(load_library().hr_set_fp32_switch(self._h, float(switch_residual),
                                                 int(stall_checks), int(max_fp32_steps)),
               "hr_set_fp32_switch")

    def reset_v(self, eta: float) -> None:
        """hr_reset_v: v = eta u at every stored point."""
        _check(load_library().hr_reset_v(self._h, float(eta)), "hr_reset_v")

    def _get(self, fn, extended: bool) -> np.ndarray:
        n = self.n_extended if extended else self.n_interior
        out = np.zeros(n)
        _check(fn(self._h, out.ctypes.data_as(_dp), n), fn.__name__)
        N0, N1, N2 = self.N
        if not extended:
            return out.reshape(N2, N1, N0)
        ng = self.NG
        if self.coords == CARTESIAN:   # the padded box: NG layers beyond every face
            return out.reshape(N2 + 2 * ng, N1 + 2 * ng, N0 + 2 * ng)
        # SinhCylindrical stores NG outer rows beyond each z face
        rows = N1 + 2 * ng if self.coords == SINHCYLINDRICAL else N1
        return out.reshape(N2, rows, N0 + ng)

    def get_u(self, extended: bool = False) -> np.ndarray:
        return self._get(load_library().hr_get_u, extended)

    def get_v(self, extended: bool = False) -> np.ndarray:
        return self._get(load_library().hr_get_v, extended)

    def _set(self, fn, a) -> None:
        a = _f64(a).reshape(-1)
        _check(fn(self._h, a.ctypes.data_as(_dp), a.size), fn.__name__)

    def set_u(self, a) -> None:
        self._set(load_library().hr_set_u, a)

    def set_v(self, a) -> None:
        self._set(load_library().hr_set_v, a)

    def residual_l2(self) -> float:
        out = ctypes.c_double()
        _check(load_library().hr_residual_l2(self._h, ctypes.byref(out)), "hr_residual_l2")
        return out.value

    def time_stage_kernels(self, eta: float, c: float = 1.0, dt: float = 0.0, n_steps: int = 50,
                           precision: int = FP64) -> np.ndarray:
        """Mean stage-kernel durations (us) for stages 1..4 and their mean, timed with
        HIP events on the grid's stream. Advances the state by n_steps."""
        out = np.zeros(5)
        _check(load_library().hr_time_stage_kernels(self._h, float(eta), float(c), float(dt),
                                                    int(n_steps), int(precision),
                                                    out.ctypes.data_as(_dp)),
               "hr_time_stage_kernels")
        return out

    def set_kernel_config(self, variant: int = 0, streaming: int = -1, chunk: int = 0,
                          graph: int = -1) -> None:
        cfg = KernelConfig(int(variant), int(streaming), int(chunk), int(graph))
        _check(load_library().hr_set_kernel_config(self._h, ctypes.byref(cfg)),
               "hr_set_kernel_config")

    def autotune(self, precision: int = FP64, n_steps: int = 5) -> tuple:
        """Times the candidate kernel configurations, keeps the fastest; returns
        (config dict, mean stage microseconds). The state is unchanged."""
        cfg = KernelConfig()
        us = ctypes.c_double()
        _check(load_library().hr_autotune(self._h, int(precision), int(n_steps), ctypes.byref(cfg),
                                          ctypes.byref(us)), "hr_autotune")
        return {"variant": cfg.variant, "streaming": cfg.streaming, "chunk": cfg.chunk,
                "graph": cfg.graph}, us.value

    def set_residual_norm(self, norm: int = NORM_POINTS, radius: float = 0.0) -> None:
        """Norm of residual_l2 and of relax's stop test: NORM_POINTS (mean of H^2
        over interior points) or NORM_VOLUME (H^2 weighted by the proper cell
        volume; radius > 0 keeps the cells whose centre lies within that
        Cartesian radius)."""
        _check(load_library().hr_set_residual_norm(self._h, int(norm), float(radius)),
               "hr_set_residual_norm")

    def set_outer_bc_order(self, order: int = 2) -> None:
        """Order (2 or 4) of the one-sided xx0 difference in the outer radiation
        condition."""
        _check(load_library().hr_set_outer_bc_order(self._h, int(order)), "hr_set_outer_bc_order")

    def set_factor_storage(self, bits: int = 32) -> None:
        """Storage of the metric factors read by the single-precision stages:
        32 (FP32 copies) or 16 (bfloat16 copies)."""
        _check(load_library().hr_set_factor_storage(self._h, int(bits)), "hr_set_factor_storage")

    def set_wait_limit(self, polls: int = 0) -> None:
        """Polls of one partner's counter before a resident-kernel wait gives up
        (0: the default, about a second); small values force the timeout path."""
        _check(load_library().hr_set_wait_limit(self._h, int(polls)), "hr_set_wait_limit")

    def set_launch_timing(self, on: bool = True) -> None:
        """Time each resident launch that later relax calls issue (HIP events
        inside the dispatch on the grid's stream); resets the totals."""
        _check(load_library().hr_set_launch_timing(self._h, 1 if on else 0),
               "hr_set_launch_timing")

    def launch_timing(self) -> dict:
        """Summed durations (us), launches and RK stages of the timed launches."""
        us = ctypes.c_double()
        nl = ctypes.c_long()
        ns = ctypes.c_long()
        _check(load_library().hr_get_launch_timing(self._h, ctypes.byref(us), ctypes.byref(nl),
                                                   ctypes.byref(ns)), "hr_get_launch_timing")
        return {"total_us": us.value, "launches": nl.value, "stages": ns.value}

    def resolved_kernel(self, precision: int = FP64) -> dict:
        """The configuration the relaxation runs in this precision, automatic
        choices resolved (variant 3 = resident kernel)."""
        cfg = KernelConfig()
        _check(load_library().hr_resolved_kernel(self._h, int(precision), ctypes.byref(cfg)),
               "hr_resolved_kernel")
        return {"variant": cfg.variant, "streaming": cfg.streaming, "chunk": cfg.chunk,
                "graph": cfg.graph}

    def kernel_config(self) -> dict:
        cfg = KernelConfig()
        _check(load_library().hr_get_kernel_config(self._h, ctypes.byref(cfg)),
               "hr_get_kernel_config")
        return {"variant": cfg.variant, "streaming": cfg.streaming, "chunk": cfg.chunk,
                "graph": cfg.graph}

    def suggest_dt(self, cfl: float = 0.5) -> float:
        out = ctypes.c_double()
        _check(load_library().hr_suggest_dt(self._h, float(cfl), ctypes.byref(out)),
               "hr_suggest_dt")
        return out.value


class Batch:
    """Many bound grids (same fd_order) relaxed together: one persistent launch per
    RK stage over every grid still relaxing, graph-captured per check interval."""

    def __init__(self, grids, stream=None):
        import torch

        L = load_library()
        self.grids = list(grids)
        arr = (ctypes.c_void_p * len(self.grids))(*[g.handle.value for g in self.grids])
        h = ctypes.c_void_p()
        _check(L.hr_batch_create(len(self.grids), arr, ctypes.byref(h)), "hr_batch_create")
        self._h = h
        dev = self.grids[0].device
        nbytes = L.hr_batch_workspace_bytes(h)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        with torch.cuda.device(dev):
            _check(L.hr_batch_bind(h, ctypes.c_void_p(aligned), nbytes,
                                   ctypes.c_void_p(self.stream.cuda_stream)), "hr_batch_bind")

    def relax(self, eta, c=1.0, n_steps: int = 1000, tol: float = 0.0, check_every: int = 100,
              precision: int = FP64, raise_on_error: bool = True) -> list:
        n = len(self.grids)
        eta = np.ascontiguousarray(np.broadcast_to(np.asarray(eta, dtype=np.float64), (n,)))
        c = np.ascontiguousarray(np.broadcast_to(np.asarray(c, dtype=np.float64), (n,)))
        cap = max(1, int(n_steps) // max(1, int(check_every)) + 2)
        hists = [np.zeros(cap) for _ in range(n)]
        reps = (RelaxReport * n)()
        for i in range(n):
            reps[i].history = hists[i].ctypes.data_as(_dp)
            reps[i].history_cap = cap
        st = load_library().hr_batch_relax(self._h, eta.ctypes.data_as(_dp), c.ctypes.data_as(_dp),
                                           int(n_steps), float(tol), int(check_every),
                                           int(precision), ctypes.cast(reps, ctypes.c_void_p))
        if st not in (OK, ENOTCONV, ENONFINITE) or (raise_on_error and st == ENONFINITE):
            _check(st, "hr_batch_relax")
        self.status = st

        def grid_status(r) -> int:
            # per grid, as hr_relax would report it: a non-finite residual first
            if r.n_history > 0 and not np.isfinite(r.residual):
                return ENONFINITE
            return OK if tol <= 0 or r.residual < tol else ENOTCONV

        return [RelaxResult(grid_status(reps[i]), reps[i].steps_taken, reps[i].fp32_steps,
                            reps[i].residual, reps[i].dt_used,
                            hists[i][:min(reps[i].n_history, cap)].copy())
                for i in range(n)]

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hr_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Module-level functions named after the C ABI entry points.
def grid_create(coords: int, N0: int, N1: int, N2: int, fd_order: int,
                params: GridParams | None = None, **kw) -> Grid:
    return Grid(coords, N0, N1, N2, fd_order, params=params, **kw)


def set_punctures(grid: Grid, m, x, P, S) -> None:
    grid.set_punctures(m, x, P, S)


def relax(grid: Grid, eta: float, c: float = 1.0, dt: float = 0.0, n_steps: int = 1000,
          tol: float = 0.0, **kw) -> RelaxResult:
    return grid.relax(eta, c, dt, n_steps, tol, **kw)


def relax_noalloc(grid: Grid, eta: float, c: float = 1.0, dt: float = 0.0,
                  n_steps: int = 1000, tol: float = 0.0, **kw) -> RelaxResult:
    return grid.relax_noalloc(eta, c, dt, n_steps, tol, **kw)


def get_u(grid: Grid, extended: bool = False) -> np.ndarray:
    return grid.get_u(extended)


def residual_l2(grid: Grid) -> float:
    return grid.residual_l2()


__all__ = ["Grid", "Batch", "GridParams", "RelaxResult", "HRError", "grid_create", "set_punctures",
           "relax", "relax_noalloc", "get_u", "residual_l2", "load_library", "default_params",
           "SINHSYMTP", "SPHERICAL", "SINHSPHERICAL", "SINHCYLINDRICAL", "CARTESIAN", "FP64", "FP32", "FP32_FP64FINISH"]
