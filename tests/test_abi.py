"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/nse_sphere.h declares, and rejects invalid arguments
synchronously (before any device work)."""
import ctypes
import os
import re

import pytest

import paper_1009_3308_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nse_sphere.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1009_3308_amd import build
        build.build()
    return pkg.lib()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nse_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert _declared_functions() == sorted(pkg.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_coeff_count_and_status_strings(L):
    assert L.nse_coeff_count(31) == 32 * 33 // 2
    assert L.nse_coeff_count(511) == 131328
    assert L.nse_coeff_count(-1) == -1
    for s in range(7):
        assert L.nse_status_string(s).decode().startswith("NSE_")


def _init(L, members, params):
    arr = (pkg.Member * len(members))(*[pkg.Member(*m) for m in members])
    h = ctypes.c_void_p(1234)
    st = L.nse_sphere_init(arr, len(members), ctypes.byref(params) if params else None, None,
                           ctypes.byref(h))
    return st, h


def _params(**kw):
    p = dict(omega=6.283, dt=1e-3, order=2, newton_iters=1, precision=0, flags=0)
    p.update(kw)
    return pkg.Params(p["omega"], p["dt"], p["order"], p["newton_iters"], p["precision"],
                      p["flags"])


@pytest.mark.parametrize("members,params,expect", [
    ([(0, 0, 1e-3)], {}, pkg.NSE_ERR_ARG),                       # N < 1
    ([(31, 0, -1.0)], {}, pkg.NSE_ERR_ARG),                      # nu < 0
    ([(31, 0, float("nan"))], {}, pkg.NSE_ERR_ARG),              # nu not finite
    ([(31, 40, 1e-3)], {}, pkg.NSE_ERR_ARG),                     # 2 nlat < 3N+2 aliases
    ([(31, -2, 1e-3)], {}, pkg.NSE_ERR_ARG),
    ([(31, 0, 1e-3)], {"order": 0}, pkg.NSE_ERR_ARG),
    ([(31, 0, 1e-3)], {"order": 6}, pkg.NSE_ERR_ARG),
    ([(31, 0, 1e-3)], {"newton_iters": 0}, pkg.NSE_ERR_ARG),
    ([(31, 0, 1e-3)], {"precision": 7}, pkg.NSE_ERR_ARG),
    ([(31, 0, 1e-3)], {"flags": 1 << 10}, pkg.NSE_ERR_ARG),
    ([(31, 0, 1e-3)], {"dt": 0.0}, pkg.NSE_ERR_ARG),
    ([(31, 0, 1e-3)], {"omega": float("inf")}, pkg.NSE_ERR_ARG),
    ([(31, 49, 1e-3)], {}, pkg.NSE_ERR_UNSUPPORTED),             # M = 98 = 2 * 7^2
    ([(31, 4000, 1e-3)], {}, pkg.NSE_ERR_UNSUPPORTED),           # M beyond the FFT limit
])
def test_invalid_arguments_rejected_before_device_work(L, members, params, expect):
    st, h = _init(L, members, _params(**params))
    assert st == expect
    assert h.value is None
    assert L.nse_last_error(None).decode() != ""


def test_null_arguments(L):
    st, h = _init(L, [(31, 0, 1e-3)], None)
    assert st == pkg.NSE_ERR_ARG
    arr = (pkg.Member * 1)(pkg.Member(31, 0, 1e-3))
    assert L.nse_sphere_init(arr, 1, ctypes.byref(_params()), None, None) == pkg.NSE_ERR_ARG
    assert L.nse_sphere_init(arr, 0, ctypes.byref(_params()), None,
                             ctypes.byref(ctypes.c_void_p())) == pkg.NSE_ERR_ARG
    for fn, args in [("nse_nonlinear", (None, None, None)), ("nse_step", (None, None, None, 0, 1)),
                     ("nse_sync", (None,)), ("nse_synthesize", (None, None, None)),
                     ("nse_analyze_velocity", (None, None, None)),
                     ("nse_nonlinear_adjoint", (None, None, None, None)),
                     ("nse_step_adjoint", (None, None, None, 0, None))]:
        assert getattr(L, fn)(*args) == pkg.NSE_ERR_ARG
    assert L.nse_sphere_destroy(None) == pkg.NSE_OK
    assert L.nse_state_count(None) == -1
