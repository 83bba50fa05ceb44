"""Plain FP64 CPU oracle for hyperbolic relaxation of puncture initial data.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``. The product package never
imports it, and it shares no code with the HIP path.

The arithmetic lives in ``hr_oracle.cpp`` (plain loops, double precision, built
with ``-ffp-contract=off`` and no fast-math); this module only marshals numpy
arrays through ctypes. What it computes follows the paper's "Basic equations"
section: Eq. (4) (Hamiltonian constraint for u with the Bowen-York source) and
Eq. (5) (the damped wave system integrated to its steady state), with the
driver order of the paper's Algorithm 1 (RHS, boundary conditions, RK substep;
residual and its L2 norm once per outer iteration).

Arrays returned by :class:`OracleGrid` are padded grid functions of shape
``(Nx2, Nx1, Nx0)`` (x0 fastest in memory), ``Nx_d = N_d + 2*NG``,
``NG = fd_order // 2``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hr_oracle.cpp")
_LIB = os.path.join(_HERE, "libhr_oracle.so")

SINHSYMTP = 0
SPHERICAL = 1
SINHSPHERICAL = 2
SINHCYLINDRICAL = 3
CARTESIAN = 4          # the cube [-rmax, rmax]^3, outer faces on all six sides

# Readings of parameters the paper leaves to its companion paper.
DEFAULT_AMAX = 1.0e6
DEFAULT_SINHWAA = 0.07
DEFAULT_RMAX = 100.0

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)
_ip = ctypes.POINTER(ctypes.c_int)


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source file with g++ (plain -O2, OpenMP, no FP
    contraction, no fast-math) into the shared library ``out``."""
    tmp = out + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-shared", "-fPIC", src, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle (``hr_oracle.cpp`` -> ``libhr_oracle.so``)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


_lib = None
_lib_path = _LIB


def use_library(path: str | None = None) -> None:
    """Load the oracle from another build of ``hr_oracle.cpp`` for the grids
    created afterwards (``None``: the default library). Used by the tests that
    plant a mistake in a copy of the source and check that a pin catches it;
    a grid keeps the library it was created with."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path if path is not None else _LIB


def lib():
    global _lib
    if _lib is None:
        if _lib_path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_lib_path)
        L.or_create.restype = ctypes.c_void_p
        L.or_create.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double] * 4
        L.or_destroy.argtypes = [ctypes.c_void_p]
        L.or_dims.argtypes = [ctypes.c_void_p, _ip]
        L.or_xx.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.or_dxx.argtypes = [ctypes.c_void_p, _dp]
        L.or_cart.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.or_metric.argtypes = [ctypes.c_void_p, _dp]
        L.or_scale_factors.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, _dp]
        L.or_to_cart.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp]
        L.or_ds_g.restype = ctypes.c_double
        L.or_ds_g.argtypes = [ctypes.c_void_p]
        L.or_suggest_dt.restype = ctypes.c_double
        L.or_suggest_dt.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.or_fd_weights.restype = ctypes.c_int
        L.or_fd_weights.argtypes = [ctypes.c_int, _dp, _dp]
        L.or_fornberg.argtypes = [ctypes.c_double, _dp, ctypes.c_int, ctypes.c_int, _dp]
        L.or_bowen_york.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, ctypes.c_long, _dp]
        L.or_set_punctures.restype = ctypes.c_int
        L.or_set_punctures.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.or_get_sources.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_bc_images.argtypes = [ctypes.c_void_p, _lp]
        L.or_set_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_get_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_fill_ghosts.argtypes = [ctypes.c_void_p, _dp]
        L.or_laplacian.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_rhs.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.or_residual.restype = ctypes.c_double
        L.or_residual.argtypes = [ctypes.c_void_p, _dp]
        L.or_residual_of.restype = ctypes.c_double
        L.or_residual_of.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_rk4_steps.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_long]
        L.or_relax.restype = ctypes.c_int
        L.or_relax.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_long, ctypes.c_double, ctypes.c_long, _dp, ctypes.c_long,
                               _lp, _lp]
        L.or_num_threads.restype = ctypes.c_int
        L.or_volume_mean.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp]
        L.or_volume_mean.restype = ctypes.c_double
        L.or_residual_volume.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.or_residual_volume.restype = ctypes.c_double
        L.or_set_bc_order.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.or_set_bc_order.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        L.or_set_num_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def fd_weights(fd_order: int):
    """Centred first- and second-derivative weights on offsets -NG..NG."""
    ng = fd_order // 2
    w1 = np.zeros(2 * ng + 1)
    w2 = np.zeros(2 * ng + 1)
    if lib().or_fd_weights(fd_order, _p(w1), _p(w2)) != 0:
        raise ValueError("unsupported fd_order")
    return w1, w2


def fornberg(z: float, x, m: int) -> np.ndarray:
    """Fornberg weights, shape (m+1, len(x))."""
    x = _f64(x)
    out = np.zeros((m + 1) * len(x))
    lib().or_fornberg(float(z), _p(x), len(x), m, _p(out))
    return out.reshape(m + 1, len(x))


def bowen_york(m, x, P, S, pts) -> np.ndarray:
    """Bowen-York A^ij at the points ``pts`` (shape (n,3)); returns (n,3,3)."""
    m = _f64(m)
    n = len(m)
    x = _f64(x).reshape(n, 3)
    P = _f64(P).reshape(n, 3)
    S = _f64(S).reshape(n, 3)
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros(len(pts) * 9)
    lib().or_bowen_york(n, _p(m), _p(x), _p(P), _p(S), _p(pts), len(pts), _p(out))
    return out.reshape(-1, 3, 3)


class OracleGrid:
    """One oracle grid: coordinates, sources, state and the relaxation loop."""

    def __init__(self, coords: int, N0: int, N1: int, N2: int, fd_order: int,
                 amax: float = DEFAULT_AMAX, sinhwaa: float = DEFAULT_SINHWAA,
                 bscale: float = 1.0, rmax: float = DEFAULT_RMAX):
        L = lib()
        self._L = L
        h = L.or_create(int(coords), N0, N1, N2, fd_order, amax, sinhwaa, bscale, rmax)
        if not h:
            raise ValueError("invalid oracle grid arguments")
        self._h = ctypes.c_void_p(h)
        self.coords = coords
        self.N = (N0, N1, N2)
        self.fd_order = fd_order
        dims = (ctypes.c_int * 4)()
        L.or_dims(self._h, dims)
        self.NG = dims[0]
        self.Nx = (dims[1], dims[2], dims[3])
        self.shape = (self.Nx[2], self.Nx[1], self.Nx[0])
        self.npad = self.Nx[0] * self.Nx[1] * self.Nx[2]

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(self, "_L", None)
        if h is not None and L is not None:
            L.or_destroy(h)
            self._h = None

    # --- geometry -------------------------------------------------------
    def xx(self, d: int) -> np.ndarray:
        out = np.zeros(self.Nx[d])
        self._L.or_xx(self._h, d, _p(out))
        return out

    def dxx(self) -> np.ndarray:
        out = np.zeros(3)
        self._L.or_dxx(self._h, _p(out))
        return out

    def cart(self):
        X = np.zeros(self.npad)
        Y = np.zeros(self.npad)
        Z = np.zeros(self.npad)
        self._L.or_cart(self._h, _p(X), _p(Y), _p(Z))
        return X.reshape(self.shape), Y.reshape(self.shape), Z.reshape(self.shape)

    def metric(self) -> dict:
        """a0,a1,a2,b0,b1,dsmin over the padded (i0,i1) plane, shape (Nx1,Nx0)."""
        n = self.Nx[0] * self.Nx[1]
        out = np.zeros(6 * n)
        self._L.or_metric(self._h, _p(out))
        names = ["a0", "a1", "a2", "b0", "b1", "dsmin"]
        return {k: out[i * n:(i + 1) * n].reshape(self.Nx[1], self.Nx[0]) for i, k in enumerate(names)}

    def scale_factors(self, x0: float, x1: float) -> np.ndarray:
        out = np.zeros(3)
        self._L.or_scale_factors(self._h, float(x0), float(x1), _p(out))
        return out

    def to_cart(self, x0: float, x1: float, x2: float) -> np.ndarray:
        out = np.zeros(3)
        self._L.or_to_cart(self._h, float(x0), float(x1), float(x2), _p(out))
        return out

    def ds_g(self) -> float:
        return self._L.or_ds_g(self._h)

    def suggest_dt(self, cfl: float = 0.5) -> float:
        return self._L.or_suggest_dt(self._h, cfl)

    def bc_images(self) -> np.ndarray:
        out = np.zeros(self.npad, dtype=np.int64)
        self._L.or_bc_images(self._h, out.ctypes.data_as(_lp))
        return out

    def interior(self, f: np.ndarray) -> np.ndarray:
        ng = self.NG
        N0, N1, N2 = self.N
        return f.reshape(self.shape)[ng:ng + N2, ng:ng + N1, ng:ng + N0]

    # --- sources and state ----------------------------------------------
    def set_punctures(self, m, x, P, S) -> None:
        m = _f64(m)
        n = len(m)
        x = _f64(x).reshape(n, 3)
        P = _f64(P).reshape(n, 3)
        S = _f64(S).reshape(n, 3)
        self._L.or_set_punctures(self._h, n, _p(m), _p(x), _p(P), _p(S))

    def sources(self):
        psi = np.zeros(self.npad)
        ssrc = np.zeros(self.npad)
        self._L.or_get_sources(self._h, _p(psi), _p(ssrc))
        return psi.reshape(self.shape), ssrc.reshape(self.shape)

    def set_state(self, u: np.ndarray, v: np.ndarray) -> None:
        u = _f64(u).reshape(-1)
        v = _f64(v).reshape(-1)
        assert u.size == self.npad and v.size == self.npad
        self._L.or_set_state(self._h, _p(u), _p(v))

    def state(self):
        u = np.zeros(self.npad)
        v = np.zeros(self.npad)
        self._L.or_get_state(self._h, _p(u), _p(v))
        return u.reshape(self.shape), v.reshape(self.shape)

    def fill_ghosts(self, f: np.ndarray) -> np.ndarray:
        f = _f64(f).reshape(-1).copy()
        self._L.or_fill_ghosts(self._h, _p(f))
        return f.reshape(self.shape)

    def pad_interior(self, f_int: np.ndarray) -> np.ndarray:
        """Embed an interior array (N2,N1,N0) into a padded one, ghosts by parity."""
        f = np.zeros(self.shape)
        self.interior(f)[...] = np.asarray(f_int, dtype=np.float64).reshape(self.N[2], self.N[1], self.N[0])
        return self.fill_ghosts(f)

    # --- operators ------------------------------------------------------
    def laplacian(self, f: np.ndarray) -> np.ndarray:
        f = _f64(f).reshape(-1)
        out = np.zeros(self.npad)
        self._L.or_laplacian(self._h, _p(f), _p(out))
        return out.reshape(self.shape)

    def rhs(self, eta: float, kappa: float, u: np.ndarray, v: np.ndarray):
        u = _f64(u).reshape(-1)
        v = _f64(v).reshape(-1)
        ku = np.zeros(self.npad)
        kv = np.zeros(self.npad)
        self._L.or_rhs(self._h, eta, kappa, _p(u), _p(v), _p(ku), _p(kv))
        return ku.reshape(self.shape), kv.reshape(self.shape)

    def residual(self, u: np.ndarray | None = None, want_H: bool = False):
        H = np.zeros(self.npad) if want_H else None
        Hp = _p(H) if want_H else None
        if u is None:
            r = self._L.or_residual(self._h, Hp)
        else:
            uu = _f64(u).reshape(-1)
            r = self._L.or_residual_of(self._h, _p(uu), Hp)
        return (r, H.reshape(self.shape)) if want_H else r

    def volume_mean(self, f: np.ndarray, radius: float = 0.0):
        """(sum f J dV / sum J dV, total volume sum J dV) over the interior cells
        whose centre lies within `radius` of the origin (all if radius <= 0),
        for a padded field f."""
        f = _f64(f).reshape(-1)
        assert f.size == self.npad
        vol = ctypes.c_double()
        m = self._L.or_volume_mean(self._h, _p(f), float(radius), ctypes.byref(vol))
        return m, vol.value

    def residual_volume(self, radius: float = 0.0) -> float:
        """Volume-weighted residual norm sqrt(sum H^2 J dV / sum J dV) of the
        state, over the cells within `radius` (all if radius <= 0)."""
        return self._L.or_residual_volume(self._h, float(radius))

    def set_bc_order(self, order: int) -> None:
        """Order (2 or 4) of the one-sided xx0 difference in the outer radiation
        condition (2 by default)."""
        if self._L.or_set_bc_order(self._h, int(order)) != 0:
            raise ValueError(f"bc order {order} not available on this grid")

    def rk4_steps(self, eta: float, kappa: float, dt: float, nsteps: int) -> None:
        self._L.or_rk4_steps(self._h, eta, kappa, dt, int(nsteps))

    def relax(self, eta: float, kappa: float, dt: float, n_steps: int, tol: float = 0.0,
              check_every: int = 100):
        """Returns (status, steps_taken, residual_history); status 0 ok,
        1 not converged, 2 non-finite."""
        cap = max(1, n_steps // max(1, check_every) + 1)
        hist = np.zeros(cap)
        st = ctypes.c_long(0)
        nh = ctypes.c_long(0)
        status = self._L.or_relax(self._h, eta, kappa, dt, int(n_steps), tol, int(check_every),
                                _p(hist), cap, ctypes.byref(st), ctypes.byref(nh))
        return status, st.value, hist[:min(nh.value, cap)].copy()


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops (for timing it on one core)."""
    lib().or_set_num_threads(int(n))
