"""ctypes binding of libmra.so: the C-ABI declared in include/mra.h.

Argument marshalling only: every computation runs in the library's gfx950
kernels.  Importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmra.so")

MRA_OK, MRA_E_ARG, MRA_E_SIZE, MRA_E_NOMEM, MRA_E_DEVICE, MRA_E_NONFINITE, MRA_E_UNSUPPORTED, MRA_E_CAPACITY = range(8)
MRA_FP64, MRA_FP32, MRA_MIXED = 0, 1, 2
MRA_FORWARD, MRA_INVERSE, MRA_PROLONG = 1, -1, 2
MRA_EXPONENTIAL, MRA_THETA_NEWTON = 0, 1
MRA_JAC_FROZEN, MRA_JAC_EXACT = 0, 1
MRA_EVAL_DENSE, MRA_EVAL_ADAPTED = 0, 1
MRA_MAX_NEWTON = 8


class GridDesc(C.Structure):
    _fields_ = [("J", C.c_int32), ("j0", C.c_int32), ("p", C.c_int32), ("adjacent_zone", C.c_int32),
                ("length", C.c_double), ("eps", C.c_double)]


class FlowDesc(C.Structure):
    _fields_ = [("nu0", C.c_double), ("cs", C.c_double), ("s0", C.c_double), ("mu", C.c_double),
                ("smag_mode", C.c_int32), ("reserved", C.c_int32)]


class SolvePtrs(C.Structure):
    _fields_ = [("omega_active", C.c_void_p), ("mask", C.c_void_p), ("index_packed", C.c_void_p),
                ("index_fine", C.c_void_p), ("n_active", C.c_void_p), ("krylov_V", C.c_void_p),
                ("hessenberg", C.c_void_p), ("scalars", C.c_void_p), ("control", C.c_void_p),
                ("capacity", C.c_int64), ("basis_stride", C.c_int64)]


EXPORTS = {
    "mra_status_str": (C.c_char_p, [C.c_int32]),
    "mra_abi_version": (C.c_int32, []),
    "mra_init": (C.c_int32, []),
    "mra_transform_ws_bytes": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.POINTER(C.c_size_t)]),
    "mra_transform": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_size_t, C.c_void_p]),
    "mra_transform_noalloc": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mra_rhs_ws_bytes": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.POINTER(C.c_size_t)]),
    "collocation_rhs": (C.c_int32, [C.POINTER(GridDesc), C.POINTER(FlowDesc), C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "collocation_rhs_adapted": (C.c_int32, [C.POINTER(GridDesc), C.POINTER(FlowDesc), C.c_int32, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mra_solve_set_evaluation": (C.c_int32, [C.c_void_p, C.c_int32]),
    "mra_solve_footprint": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "mra_solve_init": (C.c_int32, [C.POINTER(GridDesc), C.POINTER(FlowDesc), C.c_int32, C.c_int32,
                                   C.c_double, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "krylov_step": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mra_solve_footprint_cap": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.c_int32, C.c_int64,
                                            C.POINTER(C.c_size_t)]),
    "mra_solve_init_cap": (C.c_int32, [C.POINTER(GridDesc), C.POINTER(FlowDesc), C.c_int32, C.c_int32,
                                       C.c_double, C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p,
                                       C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]),
    "mra_solve_capacity": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32), C.c_void_p]),
    "mra_solve_migrate": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mra_scalar_init": (C.c_int32, [C.c_void_p, C.POINTER(GridDesc), C.c_int32, C.c_double, C.c_double,
                                    C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "solve_batch": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int32), C.c_void_p]),
    "mra_solve_read": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "mra_solve_track": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p]),
    "mra_solve_ptrs_get": (C.c_int32, [C.c_void_p, C.POINTER(SolvePtrs)]),
    "mra_solve_destroy": (C.c_int32, [C.c_void_p]),
    "mra_solve_set_integrator": (C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_void_p]),
    "mra_solve_set_jacobian": (C.c_int32, [C.c_void_p, C.c_int32]),
    "mra_scalar_set_condensation": (C.c_int32, [C.c_void_p, C.c_double, C.c_void_p]),
    "mra_tune_set_tile": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "mra_tune_get_tile": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "mra_time_kernel": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    C.POINTER(C.c_float)]),
    "mra_step_profile": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.POINTER(C.c_double),
                                     C.c_int32]),
}


def load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1604_08159_amd.build.build_library()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class MraError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {msg} (status {status})")
        self.status = status
