"""ctypes declarations of the C ABI in include/kfac_pinn.h.

Argument marshalling only: every computation happens in libkfac_pinn.so.  Loading
fails loudly when the library has not been built (there is no fallback)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkfac_pinn.so")

(KP_OK, KP_ERR_ARG, KP_ERR_OOM, KP_ERR_HIP, KP_ERR_NOT_PD, KP_ERR_NONFINITE, KP_ERR_STATE,
 KP_ERR_NOT_CONVERGED) = range(8)
KP_F64, KP_F32, KP_MIXED_BF16, KP_MIXED_F16 = 0, 1, 2, 3


class kp_problem(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("widths", C.POINTER(C.c_int32)),
                ("time_coord", C.c_int32), ("coef_time", C.c_double), ("coef_lap", C.c_double),
                ("lap_mask", C.POINTER(C.c_uint8)), ("precision", C.c_int32),
                ("max_interior", C.c_int32), ("max_boundary", C.c_int32),
                ("workspace_limit_bytes", C.c_size_t), ("op_coef", C.POINTER(C.c_double)),
                ("coef_xgrad", C.c_double), ("coef_gradsq", C.c_double),
                ("coef_const", C.c_double)]


class kp_hparams(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("beta", C.c_double), ("momentum", C.c_double),
                ("lr_mode", C.c_int32), ("lr", C.c_double), ("grid_min_exp", C.c_int32),
                ("grid_max_exp", C.c_int32)]


class kp_step_info(C.Structure):
    _fields_ = [("loss_interior", C.c_double), ("loss_boundary", C.c_double),
                ("lr_chosen", C.c_double), ("loss_after", C.c_double), ("status", C.c_int32),
                ("step", C.c_int32), ("momentum_chosen", C.c_double)]


class kp_sampler(C.Structure):
    _fields_ = [("seed_interior", C.c_uint64), ("seed_boundary", C.c_uint64),
                ("seed_initial", C.c_uint64), ("n_interior", C.c_int32),
                ("n_boundary", C.c_int32), ("n_initial", C.c_int32), ("face_lo", C.c_int32),
                ("target_kind", C.c_int32), ("scale", C.c_double), ("kappa", C.c_double)]


_V = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = {
    "kfac_pinn_create": (C.c_int, [C.POINTER(kp_problem), _V, C.POINTER(_V)]),
    "kfac_pinn_destroy": (C.c_int, [_V]),
    "kfac_pinn_reset_state": (C.c_int, [_V, C.c_int32]),
    "kfac_pinn_num_params": (C.c_int64, [C.POINTER(C.c_int32), C.c_int32]),
    "kfac_pinn_sample": (C.c_int, [_V, C.POINTER(kp_sampler), C.c_int64, _V, _V, _V, _V]),
    "kfac_pinn_forward_laplacian": (C.c_int, [_V, _V, _V, C.c_int32, _V, _V, _V]),
    "kfac_pinn_forward_laplacian_vjp": (C.c_int, [_V, _V, _V, C.c_int32, _V, _V, _V, _V, _V]),
    "kfac_pinn_factors": (C.c_int, [_V, _V, _V, _V, C.c_int32, _V, _V, C.c_int32, C.c_double,
                                    _V, _V]),
    "kfac_pinn_invert": (C.c_int, [_V, C.c_double]),
    "kfac_pinn_layer_gramian": (C.c_int, [_V, C.c_int32, C.c_int32, _V, _V]),
    "kfac_pinn_precondition": (C.c_int, [_V, _V, _V]),
    "kfac_pinn_precondition_layer_noalloc": (C.c_int, [C.c_int32, C.c_int32, _V, _V, _V, _V, _V,
                                                       _V, _V]),
    "kfac_pinn_set_max_sweeps": (C.c_int, [_V, C.c_int32]),
    "kfac_pinn_set_sweep_wait": (C.c_int, [_V, C.c_int32]),
    "kfac_pinn_check_guards": (C.c_int, [_V, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "kfac_pinn_step": (C.c_int, [_V, _V, _V, _V, C.c_int32, _V, _V, C.c_int32,
                                 C.POINTER(kp_hparams), _V]),
    "kfac_pinn_get_factor": (C.c_int, [_V, C.c_int32, C.c_int32, C.c_int32, _V]),
    "kfac_pinn_set_factor": (C.c_int, [_V, C.c_int32, C.c_int32, C.c_int32, _V]),
    "kfac_pinn_get_preconditioner": (C.c_int, [_V, C.c_int32, C.c_int32, _V, _V]),
    "kfac_pinn_get_line_search": (C.c_int, [_V, _V]),
    "kfac_pinn_get_momentum": (C.c_int, [_V, _V]),
    "kfac_pinn_set_momentum": (C.c_int, [_V, _V, C.c_int64]),
    "kfac_pinn_timing_enable": (C.c_int, [_V, C.c_int32]),
    "kfac_pinn_timing_read": (C.c_int, [_V, C.POINTER(C.c_double)]),
    "kfac_pinn_get_sweeps": (C.c_int, [_V, C.POINTER(C.c_int32)]),
    "kfac_pinn_set_line_search_lanes": (C.c_int, [_V, C.c_int32]),
    "kfac_pinn_get_workspace": (C.c_int, [_V, C.POINTER(C.c_int32)]),
    "kfac_pinn_batch_create": (C.c_int, [C.POINTER(kp_problem), C.c_int32, _V, C.POINTER(_V)]),
    "kfac_pinn_batch_destroy": (C.c_int, [_V]),
    "kfac_pinn_batch_context": (C.c_int, [_V, C.c_int32, C.POINTER(_V)]),
    "kfac_pinn_batch_set_graph": (C.c_int, [_V, C.c_int32]),
    "kfac_pinn_batch_set_grouped": (C.c_int, [_V, C.c_int32]),
    "kfac_pinn_batch_is_grouped": (C.c_int, [_V, C.POINTER(C.c_int32)]),
    "kfac_pinn_batch_tune": (C.c_int, [_V, C.POINTER(_V), C.POINTER(_V), C.POINTER(_V),
                                       C.POINTER(C.c_int32), C.POINTER(_V), C.POINTER(_V),
                                       C.POINTER(C.c_int32), C.c_char_p,
                                       C.POINTER(C.c_int32)]),
    "kfac_pinn_batch_get_sweeps": (C.c_int, [_V, C.c_int32, C.POINTER(C.c_int32)]),
    "kfac_pinn_batch_step": (C.c_int, [_V, C.POINTER(_V), C.POINTER(_V), C.POINTER(_V),
                                       C.POINTER(C.c_int32), C.POINTER(_V), C.POINTER(_V),
                                       C.POINTER(C.c_int32), C.POINTER(kp_hparams), _V]),
    "kfac_pinn_sync": (C.c_int, [_V]),
    "kfac_pinn_status_string": (C.c_char_p, [C.c_int]),
    "kfac_pinn_last_error": (C.c_char_p, []),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__; __graft_entry__.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class KfacPinnError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.kfac_pinn_status_string(status).decode()
        detail = L.kfac_pinn_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")
        self.status = status


def check(status: int, where: str) -> None:
    if status != KP_OK:
        raise KfacPinnError(status, where)
