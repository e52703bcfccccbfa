"""ctypes binding of the C ABI declared in include/ins.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libins.so")

INS_OK = 0
INS_ERR_INVALID = -1
INS_ERR_UNSUPPORTED = -2
INS_ERR_OOM = -3
INS_ERR_HIP = -4
INS_FP64 = 0
INS_FP32 = 1
INS_FP32_ALL = 2
INS_BC_PERIODIC = 0
INS_BC_WALLS_Y = 1
INS_RK4 = 0
INS_WRAY3 = 1
INS_PRESSURE_AUTO = 0
INS_PRESSURE_FFT = 1
INS_PRESSURE_CG = 2

_STATUS_NAMES = {
    INS_ERR_INVALID: "INS_ERR_INVALID",
    INS_ERR_UNSUPPORTED: "INS_ERR_UNSUPPORTED",
    INS_ERR_OOM: "INS_ERR_OOM",
    INS_ERR_HIP: "INS_ERR_HIP",
}


class InsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("n", C.c_int64 * 3),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("batch", C.c_int64),
    ]


_P = C.c_void_p
_D = C.c_double
_SIGS = {
    "ins_create": ([C.POINTER(Grid), C.c_int, _D, C.c_int, C.POINTER(_P)]),
    "ins_destroy": ([_P]),
    "ins_set_stream": ([_P, _P]),
    "ins_workspace_bytes": ([_P, C.POINTER(C.c_size_t)]),
    "ins_rhs": ([_P, _P, _P]),
    "ins_divergence": ([_P, _P, _P]),
    "ins_gradient": ([_P, _P, _P]),
    "ins_poisson_solve": ([_P, _P, _P]),
    "ins_project": ([_P, _P, _P, _P]),
    "ins_step_rk4": ([_P, _P, _P, _D]),
    "ins_rhs_vjp": ([_P, _P, _P, _P]),
    "ins_divergence_vjp": ([_P, _P, _P]),
    "ins_gradient_vjp": ([_P, _P, _P]),
    "ins_poisson_solve_vjp": ([_P, _P, _P]),
    "ins_project_vjp": ([_P, _P, _P]),
    "ins_step_rk4_vjp": ([_P, _P, _P, _P, _D]),
    "ins_step_wray3": ([_P, _P, _P, _D]),
    "ins_step_wray3_vjp": ([_P, _P, _P, _P, _D]),
    "ins_step_save": ([_P, C.c_int, _P, _P, _D, _P, _P]),
    "ins_cg_set": ([_P, _D, C.c_int, C.c_int]),
    "ins_set_y_faces": ([_P, C.POINTER(C.c_double)]),
    "ins_set_faces": ([_P, C.c_int, C.POINTER(C.c_double)]),
    "ins_cg_info": ([_P, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "ins_set_pressure_solver": ([_P, C.c_int]),
    "ins_set_body_force": ([_P, C.POINTER(C.c_double)]),
    "ins_get_pressure_solver": ([_P, C.POINTER(C.c_int)]),
    "ins_step_vjp_saved": ([_P, C.c_int, _P, _P, _P, _P, _P, _D]),
    "ins_scheme_stage_count": ([C.c_int]),
    "ins_eddy_set": ([_P, _D, _D]),
    "ins_eddy_forward": ([_P, _P, _P]),
    "ins_eddy_backward": ([_P, _P, _P, _P]),
    "ins_closure_set": ([_P, _P]),
    "ins_closure_grad": ([_P, _P]),
    "ins_cnn_forward": ([_P, _P, _P]),
    "ins_cnn_backward": ([_P, _P, _P, _P, _P]),
    "ins_cnn_saved": ([_P, C.c_int, _P]),
    "ins_face_filter": ([_P, _P, C.c_int, _P]),
    "ins_energy_spectrum": ([_P, _P, _P, C.c_int]),
    "ins_stats": ([_P, _P, C.POINTER(_D)]),
    "ins_stats_noalloc": ([_P, _P, _P]),
    "ins_stream_copy": ([_P, _P, _P, C.c_size_t]),
    "ins_profile_enable": ([_P, C.c_int]),
    "ins_profile_reset": ([_P]),
    "ins_profile_count": ([_P, C.POINTER(C.c_int)]),
    "ins_profile_read": ([_P, C.c_int, C.c_char_p, C.c_size_t, C.POINTER(C.c_int64), C.POINTER(_D)]),
}

_lib = None


def load():
    """Load libins.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first (python -m paper_2604_18536_amd.build)"
        )
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.ins_last_error.argtypes = []
    lib.ins_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def check(status):
    if status != INS_OK:
        msg = load().ins_last_error()
        raise InsError(status, msg.decode() if msg else "")
    return status


def call(name, *args):
    return check(getattr(load(), name)(*args))
