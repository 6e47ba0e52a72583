"""ctypes binding of librlb.so (the C ABI in include/rlb.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librlb.so")

RLB_OK, RLB_EINVAL, RLB_ENOMEM, RLB_EDEVICE, RLB_EUNPHYSICAL = 0, -1, -2, -3, -4
BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2
F64, F32, F32DEV, F16DEV, BF16DEV = 0, 1, 2, 3, 4
COLLIDE_AUTO, COLLIDE_F32, COLLIDE_F64, COLLIDE_F32_MOM64 = 0, 1, 2, 3

# Every symbol include/rlb.h declares (checked by the tests).
EXPORTS = (
    "rlb_buffer_layout", "rlb_init", "rlb_step", "rlb_step_g", "rlb_current", "rlb_moments",
    "rlb_fields_g", "rlb_counters", "rlb_adjoint_step", "rlb_moments_adjoint", "rlb_init_adjoint",
    "rlb_destroy", "rlb_status_string", "rlb_last_error", "rlb_advance_g", "rlb_trajectory_g",
    "rlb_adjoint_sweep", "rlb_adjoint_flush", "rlb_set_tau_field", "rlb_hold_eta_over_s",
    "rlb_transport", "rlb_adjoint_flush_tau_field", "rlb_moments_noalloc", "rlb_adjoint_segment",
    "rlb_lam_gather", "rlb_encode16",
)
LAM_IN_READER, LAM_OUT_READER = 1, 2


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("c_l", ctypes.c_double),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("inflow_n", ctypes.c_double), ("inflow_e", ctypes.c_double),
        ("inflow_beta", ctypes.c_double * 3),
        ("storage", ctypes.c_int32),
        ("n_ref", ctypes.c_double), ("e_ref", ctypes.c_double),
        ("collide", ctypes.c_int32),
        ("kappa", ctypes.c_double),
        ("inplace", ctypes.c_int32),
    ]


class RLBError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({detail})")


class UnphysicalState(RLBError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.rlb_buffer_layout.argtypes = [ctypes.POINTER(Params), i64p, i64p]
    L.rlb_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_double),
                           vp, vp, vp, vp, vp, vp, vp]
    L.rlb_step.argtypes = [vp, ctypes.c_int32]
    L.rlb_step_g.argtypes = [vp, vp, vp]
    L.rlb_current.argtypes = [vp, ctypes.POINTER(vp)]
    L.rlb_moments.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.rlb_moments_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.rlb_fields_g.argtypes = [vp, vp, vp, vp]
    L.rlb_counters.argtypes = [vp, i64p]
    L.rlb_adjoint_step.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.rlb_advance_g.argtypes = [vp, vp, vp, vp, ctypes.c_int32]
    L.rlb_trajectory_g.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32]
    L.rlb_adjoint_sweep.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp,
                                    ctypes.POINTER(vp)]
    L.rlb_adjoint_flush.argtypes = [vp, vp, vp, vp]
    L.rlb_adjoint_segment.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp,
                                      ctypes.c_int32, ctypes.POINTER(vp)]
    L.rlb_lam_gather.argtypes = [vp, vp, vp]
    L.rlb_encode16.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int64, vp]
    L.rlb_set_tau_field.argtypes = [vp, vp]
    L.rlb_hold_eta_over_s.argtypes = [vp, ctypes.c_double, ctypes.c_double]
    L.rlb_transport.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp]
    L.rlb_adjoint_flush_tau_field.argtypes = [vp, vp]
    L.rlb_moments_adjoint.argtypes = [vp, vp, vp, vp, vp]
    L.rlb_init_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.rlb_destroy.argtypes = [vp]
    L.rlb_status_string.argtypes = [ctypes.c_int]
    L.rlb_status_string.restype = ctypes.c_char_p
    L.rlb_last_error.argtypes = []
    L.rlb_last_error.restype = ctypes.c_char_p
    for name in ("rlb_buffer_layout", "rlb_init", "rlb_step", "rlb_step_g", "rlb_current",
                 "rlb_moments", "rlb_fields_g", "rlb_counters", "rlb_adjoint_step", "rlb_moments_adjoint",
                 "rlb_init_adjoint", "rlb_destroy", "rlb_advance_g", "rlb_trajectory_g",
                 "rlb_adjoint_sweep", "rlb_adjoint_flush", "rlb_set_tau_field",
                 "rlb_hold_eta_over_s", "rlb_transport", "rlb_adjoint_flush_tau_field",
                 "rlb_moments_noalloc", "rlb_adjoint_segment", "rlb_lam_gather", "rlb_encode16"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().rlb_status_string(int(s)).decode()


def check(status: int, where: str):
    if status == RLB_OK:
        return
    detail = lib().rlb_last_error().decode()
    if status == RLB_EUNPHYSICAL:
        raise UnphysicalState(status, where, detail)
    raise RLBError(status, where, detail)
