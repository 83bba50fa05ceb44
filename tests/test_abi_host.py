"""CPU-side checks of the C ABI library: it loads, exports every symbol the
header declares, validates arguments and computes its host-side geometry
(no device calls are made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2501_14030_amd as hr
from paper_2501_14030_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hrelax.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return hr.load_library()


def test_library_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # and the bindings wrap every one of them
    from paper_2501_14030_amd import mlp
    assert set(names) <= set(hr._SIGNATURES) | set(mlp._SIG)


def _create(lib, coords, N0, N1, N2, order, params=None):
    h = ctypes.c_void_p()
    pp = ctypes.byref(params) if params is not None else None
    st = lib.hr_grid_create(coords, N0, N1, N2, order, pp, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("args", [
    (0, 32, 16, 5, 8),     # odd N2
    (0, 3, 16, 4, 8),      # N0 < NG
    (0, 32, 3, 4, 8),      # N1 < NG
    (0, 32, 16, 4, 7),     # odd order
    (0, 32, 16, 4, 12),    # unsupported order
    (5, 32, 16, 4, 8),     # unknown coordinates
    (0, 32, 16, 0, 8),
    (4, 32, 16, 3, 8),     # Cartesian N2 < NG
    (4, 1, 16, 8, 2),      # Cartesian N0 < 2
])
def test_create_rejects_invalid_arguments(lib, args):
    st, h = _create(lib, *args)
    assert st == hr.EINVAL and not h.value
    assert len(lib.hr_last_error()) > 0


def test_create_rejects_bad_params(lib):
    p = hr.default_params(sinhwaa=-1.0)
    st, h = _create(lib, 0, 16, 8, 4, 8, p)
    assert st == hr.EINVAL


def test_workspace_and_sizes(lib):
    st, h = _create(lib, 0, 128, 128, 16, 10)
    assert st == hr.OK
    ni = ctypes.c_size_t()
    ne = ctypes.c_size_t()
    assert lib.hr_grid_sizes(h, ctypes.byref(ni), ctypes.byref(ne)) == hr.OK
    assert ni.value == 128 * 128 * 16
    assert ne.value == 133 * 128 * 16
    ws = lib.hr_workspace_bytes(h)
    # 10 FP64 grid functions and 14 FP32 ones (10 + the split-state base slopes,
    # base p and S_src p^-7) dominate
    per_point = 10 * 8 + 14 * 4
    assert per_point * ne.value <= ws < per_point * ne.value * 1.1
    # calls that need a bound device workspace refuse politely
    out = ctypes.c_double()
    assert lib.hr_residual_l2(h, ctypes.byref(out)) == hr.ESTATE
    lib.hr_grid_destroy(h)
    lib.hr_grid_destroy(None)


@pytest.mark.parametrize("spec", [
    workloads.GridSpec(0, 32, 16, 4, 8, bscale=1.0),
    workloads.GridSpec(0, 128, 128, 16, 10, bscale=5.0),
    workloads.GridSpec(1, 128, 64, 8, 10, rmax=100.0),
    workloads.GridSpec(2, 64, 32, 8, 10),
    workloads.GridSpec(3, 32, 16, 4, 8, amax=10.0, sinhwaa=0.3),
    workloads.GridSpec(3, 37, 22, 6, 10, amax=1.0e3, sinhwaa=0.15),
    workloads.GridSpec(4, 24, 20, 16, 8, rmax=6.0),
    workloads.GridSpec(4, 70, 13, 11, 10, rmax=5.0),
])
def test_suggested_dt_matches_oracle(lib, oracle_lib, spec):
    p = hr.default_params(amax=spec.amax, sinhwaa=spec.sinhwaa, bscale=spec.bscale,
                          rmax=spec.rmax)
    st, h = _create(lib, spec.coords, spec.N0, spec.N1, spec.N2, spec.fd_order, p)
    assert st == hr.OK
    dt = ctypes.c_double()
    assert lib.hr_suggest_dt(h, 0.5, ctypes.byref(dt)) == hr.OK
    og = oracle_lib.OracleGrid(spec.coords, spec.N0, spec.N1, spec.N2, spec.fd_order,
                               amax=spec.amax, sinhwaa=spec.sinhwaa, bscale=spec.bscale,
                               rmax=spec.rmax)
    np.testing.assert_allclose(dt.value, og.suggest_dt(0.5), rtol=1e-15)
    lib.hr_grid_destroy(h)


def test_residual_norm_arguments_on_an_unbound_grid(lib):
    """hr_set_residual_norm validates its arguments on the host (no device
    call on a grid that is not bound)."""
    p = hr.default_params(rmax=2.0)
    st, h = _create(lib, 1, 20, 14, 6, 8, p)
    assert st == hr.OK
    f = lib.hr_set_residual_norm
    assert f(h, hr.NORM_VOLUME, 0.0) == hr.OK
    assert f(h, hr.NORM_VOLUME, 1.0) == hr.OK            # cells with r < 1 kept
    assert f(h, hr.NORM_VOLUME, 1e-6) == hr.EINVAL       # no cell centre inside
    assert f(h, hr.NORM_POINTS, 1.0) == hr.EINVAL        # radius needs the volume norm
    assert f(h, hr.NORM_VOLUME, float("inf")) == hr.EINVAL
    assert f(h, 7, 0.0) == hr.EINVAL
    assert f(None, hr.NORM_POINTS, 0.0) == hr.EINVAL
    assert f(h, hr.NORM_POINTS, 0.0) == hr.OK
    lib.hr_grid_destroy(h)


def test_cartesian_sizes_and_host_refusals(lib):
    """A Cartesian grid stores the padded box; its host-side refusals (the
    volume norm, a fourth-order face difference across a face with fewer than
    four points) need no device."""
    st, h = _create(lib, 4, 24, 20, 16, 8, hr.default_params(rmax=6.0))
    assert st == hr.OK
    ni = ctypes.c_size_t()
    ne = ctypes.c_size_t()
    assert lib.hr_grid_sizes(h, ctypes.byref(ni), ctypes.byref(ne)) == hr.OK
    assert ni.value == 24 * 20 * 16 and ne.value == 32 * 28 * 24
    assert lib.hr_set_residual_norm(h, hr.NORM_VOLUME, 0.0) == hr.EINVAL
    assert lib.hr_set_residual_norm(h, hr.NORM_POINTS, 0.0) == hr.OK
    assert lib.hr_set_outer_bc_order(h, 4) == hr.OK
    lib.hr_grid_destroy(h)
    st, h = _create(lib, 4, 8, 8, 3, 2, hr.default_params(rmax=1.0))   # N2 = 3
    assert st == hr.OK
    assert lib.hr_set_outer_bc_order(h, 4) == hr.EINVAL
    assert lib.hr_set_outer_bc_order(h, 2) == hr.OK
    lib.hr_grid_destroy(h)
    st, h = _create(lib, 4, 8, 8, 8, 2, hr.default_params(rmax=-1.0))
    assert st == hr.EINVAL
    # a puncture on a cell centre (r = 0 there) is refused before any device
    # call; one between centres passes the argument checks (ESTATE: unbound)
    st, h = _create(lib, 4, 8, 8, 8, 2, hr.default_params(rmax=4.0))   # centres at +-0.5, ...
    assert st == hr.OK
    m = np.array([0.5])
    zero = np.zeros(3)
    dp = ctypes.POINTER(ctypes.c_double)

    def put(x):
        x = np.asarray(x, dtype=np.float64)
        return lib.hr_set_punctures(h, 1, m.ctypes.data_as(dp), x.ctypes.data_as(dp),
                                    zero.ctypes.data_as(dp), zero.ctypes.data_as(dp))

    assert put([0.5, -1.5, 2.5]) == hr.EINVAL
    assert put([0.5, -1.5, 2.0]) == hr.ESTATE
    lib.hr_grid_destroy(h)


def test_outer_bc_order_arguments(lib):
    p = hr.default_params(rmax=2.0)
    st, h = _create(lib, 1, 20, 14, 6, 8, p)
    assert st == hr.OK
    f = lib.hr_set_outer_bc_order
    assert f(h, 4) == hr.OK and f(h, 2) == hr.OK
    for bad in (0, 1, 3, 6):
        assert f(h, bad) == hr.EINVAL
    assert f(None, 2) == hr.EINVAL
    lib.hr_grid_destroy(h)
    st, h = _create(lib, 1, 3, 14, 6, 4, p)          # N0 = 3 < 4
    assert st == hr.OK
    assert lib.hr_set_outer_bc_order(h, 4) == hr.EINVAL
    assert lib.hr_set_outer_bc_order(h, 2) == hr.OK
    lib.hr_grid_destroy(h)


def test_factor_storage_arguments(lib):
    st, h = _create(lib, 0, 32, 16, 4, 8, hr.default_params(bscale=1.0))
    assert st == hr.OK
    f = lib.hr_set_factor_storage
    assert f(h, 16) == hr.OK and f(h, 32) == hr.OK
    for bad in (0, 8, 64):
        assert f(h, bad) == hr.EINVAL
    assert f(None, 32) == hr.EINVAL
    lib.hr_grid_destroy(h)


def test_missing_library_fails_loudly(tmp_path):
    """The binding has no fallback: loading a library that is not there raises
    with a message that names the build step (run in a child process so that
    this process's loaded library is untouched)."""
    import subprocess
    import sys
    code = ("import paper_2501_14030_amd as hr\n"
            "try:\n"
            f"    hr.load_library({str(tmp_path / 'libhrelax.so')!r})\n"
            "except Exception as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    print('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=300)
    assert "raised:" in r.stdout and "missing" in r.stdout, r.stdout + r.stderr


def test_sinhsymtp_punctures_must_sit_at_the_foci(lib):
    """hr_set_punctures checks its arguments before the grid's state: on a
    SinhSymTP grid a puncture off the foci (0, 0, +-bscale) is HR_EINVAL (the
    coordinates concentrate resolution there); on the foci, or on a Spherical
    grid anywhere, the arguments pass and the unbound grid gives HR_ESTATE."""
    b = 2.5
    st, h = _create(lib, 0, 16, 8, 4, 8, hr.default_params(bscale=b))
    assert st == hr.OK
    dp = ctypes.POINTER(ctypes.c_double)

    def call(handle, xs):
        n = len(xs)
        m = np.full(n, 0.5)
        x = np.ascontiguousarray(np.asarray(xs, dtype=np.float64).reshape(n, 3))
        z = np.zeros((n, 3))
        return lib.hr_set_punctures(handle, n, m.ctypes.data_as(dp), x.ctypes.data_as(dp),
                                    z.ctypes.data_as(dp), z.ctypes.data_as(dp))

    assert call(h, [[0, 0, b], [0, 0, -b]]) == hr.ESTATE
    assert call(h, [[0, 0, -b]]) == hr.ESTATE
    assert call(h, [[0, 0, b * (1 + 5e-13)]]) == hr.ESTATE      # within 1e-12 bscale
    for bad in ([[0, 0, b * (1 + 1e-9)]], [[0, 0, 0]], [[1e-6, 0, b]], [[0, 1e-6, -b]],
                [[0, 0, b], [0, 0, 0.5 * b]]):
        assert call(h, bad) == hr.EINVAL, bad
        assert "foci" in lib.hr_last_error().decode()
    lib.hr_grid_destroy(h)
    st, h = _create(lib, 1, 16, 8, 4, 8, hr.default_params(rmax=10.0))
    assert st == hr.OK
    assert call(h, [[0.3, -0.2, 0.7]]) == hr.ESTATE
    lib.hr_grid_destroy(h)
