"""Host-side checks of the C ABI library (no GPU needed): it loads and exports
every entry point that include/kfac_pinn.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kfac_pinn.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(kfac_pinn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_named_calls():
    names = declared()
    for n in ("kfac_pinn_forward_laplacian", "kfac_pinn_factors", "kfac_pinn_invert",
              "kfac_pinn_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_15603_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("libkfac_pinn.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared()) == set(_native.EXPORTED)


def test_num_params_without_gpu():
    from paper_2405_15603_amd import _native
    L = _native.lib()
    w = (ctypes.c_int32 * 6)(100, 768, 768, 512, 512, 1)
    assert L.kfac_pinn_num_params(w, 5) == 1325057
    assert L.kfac_pinn_status_string(4).decode().startswith("damped factor")


def test_create_rejects_bad_arguments_before_touching_the_device():
    """Argument errors are reported synchronously (KP_ERR_ARG) without HIP calls."""
    from paper_2405_15603_amd import _native as N
    L = N.lib()
    w = (ctypes.c_int32 * 3)(2, 8, 3)      # scalar output required
    prob = N.kp_problem(2, w, -1, 0.0, -1.0, None, N.KP_F32, 10, 10, 0)
    h = ctypes.c_void_p()
    assert L.kfac_pinn_create(ctypes.byref(prob), None, ctypes.byref(h)) == N.KP_ERR_ARG
    assert "scalar" in L.kfac_pinn_last_error().decode()
    w = (ctypes.c_int32 * 3)(2, 8, 1)
    prob = N.kp_problem(2, w, -1, 0.0, -1.0, None, 7, 10, 10, 0)
    assert L.kfac_pinn_create(ctypes.byref(prob), None, ctypes.byref(h)) == N.KP_ERR_ARG


def test_create_rejects_bad_operator_coefficients():
    """A coefficient matrix must be symmetric and finite, comes instead of a mask,
    and with a time term leaves the time coordinate out of the second-order part."""
    from paper_2405_15603_amd import _native as N
    L = N.lib()
    w = (ctypes.c_int32 * 3)(3, 8, 1)
    h = ctypes.c_void_p()

    def create(coef, time_coord=-1, c_t=0.0, mask=None):
        cf = (ctypes.c_double * 9)(*coef)
        prob = N.kp_problem(2, w, time_coord, c_t, -1.0, mask, N.KP_F64, 10, 10, 0, cf)
        return L.kfac_pinn_create(ctypes.byref(prob), None, ctypes.byref(h))

    assert create([1, 2, 0, 0, 1, 0, 0, 0, 1]) == N.KP_ERR_ARG
    assert "symmetric" in L.kfac_pinn_last_error().decode()
    assert create([1, 0, 0, 0, float("nan"), 0, 0, 0, 1]) == N.KP_ERR_ARG
    assert create([1, 0, 0, 0, 1, 0.5, 0, 0.5, 1], time_coord=0, c_t=1.0) == N.KP_ERR_ARG
    assert "time coordinate" in L.kfac_pinn_last_error().decode()
    m = (ctypes.c_uint8 * 3)(1, 1, 1)
    assert create([1, 0, 0, 0, 1, 0, 0, 0, 1], mask=m) == N.KP_ERR_ARG
