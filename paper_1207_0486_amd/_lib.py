"""ctypes bindings of the hns C ABI (include/hns.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhns.so")

HNS_OK = 0
HNS_NOT_CONVERGED = 1
HNS_ERR_INVALID = -1
HNS_ERR_HIP = -2
HNS_ERR_OOM = -3
HNS_ERR_MESH = -4
HNS_ERR_BREAKDOWN = -5

HNS_POISSON = 0x1
HNS_HELMHOLTZ = 0x2
HNS_KEEP_FP32 = 0x10
HNS_STEP_AUX = 0x20
HNS_GPU_ASSEMBLY = 0x40
HNS_KEEP_HOST = 0x80
HNS_FMT_AUTO = 0x000
HNS_FMT_CSR = 0x100
HNS_FMT_SELL = 0x200
HNS_FMT_SDIA = 0x400
HNS_MATRIX_FREE = 0x800

HNS_FP64 = 0
HNS_MIXED = 1


class hns_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_tets", C.c_int64), ("tets", C.POINTER(C.c_int32)),
                ("bc", C.POINTER(C.c_uint8)),
                ("n_surf_tris", C.c_int64), ("surf_tris", C.POINTER(C.c_int32))]


class hns_hex_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_hex", C.c_int64), ("order", C.c_int32), ("reserved", C.c_int32),
                ("hex", C.POINTER(C.c_int32)), ("bc", C.POINTER(C.c_uint8))]


class hns_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer_iterations", C.c_int32),
                ("relres_true", C.c_double), ("removed_mean", C.c_double),
                ("status", C.c_int32), ("reserved", C.c_int32)]


# every exported function with its argument and result types
_SIGNATURES = {
    "hns_assemble": (C.c_int, [C.POINTER(hns_mesh), C.c_double, C.c_double, C.c_double,
                               C.c_uint32, C.POINTER(C.c_void_p)]),
    "hns_assemble_hex": (C.c_int, [C.POINTER(hns_hex_mesh), C.c_double, C.c_double,
                                   C.c_double, C.c_uint32, C.POINTER(C.c_void_p)]),
    "hns_solve": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                            C.c_uint32, C.c_void_p, C.POINTER(hns_solve_info)]),
    "hns_solve_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_int, C.c_uint32, C.c_void_p,
                                    C.POINTER(hns_solve_info)]),
    "hns_noalloc_bytes": (C.c_size_t, [C.c_void_p, C.c_uint32]),
    "hns_noalloc_scratch_bytes": (C.c_size_t, []),
    "hns_solve_batched": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.c_void_p,
                                    C.c_void_p, C.c_double, C.c_int, C.c_uint32, C.c_void_p,
                                    C.POINTER(hns_solve_info)]),
    "hns_tune_batched": (C.c_int, [C.c_void_p, C.c_int, C.c_uint32, C.c_void_p,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "hns_batch_footprint": (C.c_size_t, [C.c_void_p, C.c_int, C.c_uint32]),
    "hns_batch_open": (C.c_int, [C.c_void_p, C.c_int, C.c_uint32, C.POINTER(C.c_void_p)]),
    "hns_batch_close": (None, [C.c_void_p]),
    "hns_batch_add": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_void_p), C.POINTER(C.c_double),
                                C.POINTER(C.c_int), C.c_void_p]),
    "hns_batch_advance": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_int)]),
    "hns_batch_poll": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(hns_solve_info),
                                 C.c_void_p]),
    "hns_batch_take": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(hns_solve_info),
                                 C.c_void_p]),
    "hns_footprint_bytes": (C.c_size_t, [C.c_void_p, C.c_int, C.c_uint32, C.c_int]),
    "hns_operator_n": (C.c_int64, [C.c_void_p]),
    "hns_operator_nnz": (C.c_int64, [C.c_void_p]),
    "hns_operator_format": (C.c_uint32, [C.c_void_p]),
    "hns_operator_ndiag": (C.c_int, [C.c_void_p]),
    "hns_operator_line_len": (C.c_int, [C.c_void_p]),
    "hns_operator_assembly": (C.c_int, [C.c_void_p]),
    "hns_set_param": (C.c_int, [C.c_void_p, C.c_char_p, C.c_double]),
    "hns_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hns_step_velocity_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]),
    "hns_step_pressure_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hns_step_correct": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "hns_apply_aux": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hns_step_advection": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hns_step_velocity_rhs_bdf": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                            C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hns_step_pressure_rhs_tau": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "hns_step_correct_rhs": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]),
    "hns_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "hns_profile_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                   C.POINTER(C.c_int64)]),
    "hns_operator_destroy": (None, [C.c_void_p]),
    "hns_status_string": (C.c_char_p, [C.c_int]),
    "hns_last_error": (C.c_char_p, []),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """Load libhns.so (built in-tree by paper_1207_0486_amd.build); fails loudly."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is missing: build it with `python paper_1207_0486_amd/build.py` "
                "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return sorted(_SIGNATURES)
