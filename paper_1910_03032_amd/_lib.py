"""ctypes declarations of the C ABI in include/sfem.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfem.so")

SFEM_OK = 0
SFEM_NOCONV = 1
APPLY_NOALLOC_MAX_BYTES = 64 << 20  # SFEM_APPLY_NOALLOC_MAX_BYTES
STATUS_NAMES = {
    0: "SFEM_OK", 1: "SFEM_NOCONV", -1: "SFEM_E_ARG", -2: "SFEM_E_MESH", -3: "SFEM_E_HIP",
    -4: "SFEM_E_NOMEM", -5: "SFEM_E_UNSUPPORTED", -6: "SFEM_E_NAN", -7: "SFEM_E_BREAKDOWN",
    -8: "SFEM_E_STATE",
}
F64, F32 = 0, 1
PRECOND_JACOBI, PRECOND_COLLOCATED_MASS, PRECOND_LOR, PRECOND_LOR32 = 0, 1, 2, 3
LOR_MAX_LEVELS = 12
MASS, DIFFUSION, HELMHOLTZ = 0, 1, 2
WEAK_GRADIENT, WEAK_CURL, WEAK_DIVERGENCE = 1, 2, 3

EXPORTED = [
    "sfem_abi_version", "sfem_create", "sfem_destroy", "sfem_set_stream", "sfem_last_error",
    "sfem_setup", "sfem_qpoint_coords", "sfem_set_coeffs", "sfem_apply", "sfem_diagonal",
    "sfem_load", "sfem_collocated_mass", "sfem_pcg", "sfem_grad_nu", "sfem_get_info",
    "sfem_setup_pressure", "sfem_stokes_apply", "sfem_convection", "sfem_weak_op", "sfem_lincomb",
    "sfem_apply_noalloc", "sfem_bdf_ext_weights", "sfem_flow_create", "sfem_flow_destroy",
    "sfem_flow_last_error", "sfem_flow_set_stream", "sfem_flow_step", "sfem_lor_setup",
    "sfem_lor_apply", "sfem_lor_vcycle",
]


class PcgOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int), ("mode", C.c_int),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int), ("check_every", C.c_int),
                ("x0_zero", C.c_int), ("precond", C.c_int), ("nullspace", C.c_int)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer", C.c_int), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("status", C.c_int)]


class CtxInfo(C.Structure):
    _fields_ = [("p", C.c_int), ("q", C.c_int), ("nelem", C.c_int64), ("ndof", C.c_int64),
                ("compact", C.c_int), ("nfields", C.c_int), ("device_bytes", C.c_int64),
                ("nassembled", C.c_int64), ("nentries", C.c_int64)]


class FlowOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("nu", C.c_double), ("rtol", C.c_double), ("order", C.c_int),
                ("pressure_mode", C.c_int), ("check_every", C.c_int), ("maxit", C.c_int),
                ("pressure_precond", C.c_int), ("velocity_mode", C.c_int)]


class FlowInfo(C.Structure):
    _fields_ = [("order", C.c_int), ("pressure", PcgInfo), ("velocity", PcgInfo * 3)]


class LorInfo(C.Structure):
    _fields_ = [("levels", C.c_int), ("rows", C.c_int64 * LOR_MAX_LEVELS),
                ("nnz", C.c_int64 * LOR_MAX_LEVELS), ("setup_ms", C.c_double),
                ("sliced", C.c_int32 * LOR_MAX_LEVELS)]


class SfemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libsfem.so (built in-tree).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1910_03032_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "sfem_abi_version": (i32, []),
        "sfem_create": (i32, [i32, vp, C.POINTER(vp)]),
        "sfem_destroy": (None, [vp]),
        "sfem_set_stream": (i32, [vp, vp]),
        "sfem_last_error": (C.c_char_p, [vp]),
        "sfem_setup": (i32, [vp, i32, i32, i64, vp, vp, i64, vp]),
        "sfem_qpoint_coords": (i32, [vp, vp]),
        "sfem_set_coeffs": (i32, [vp, dbl, dbl, vp, i32]),
        "sfem_apply": (i32, [vp, i32, i32, i32, vp, vp]),
        "sfem_apply_noalloc": (i32, [vp, i32, i32, i32, vp, vp]),
        "sfem_diagonal": (i32, [vp, i32, i32, vp]),
        "sfem_load": (i32, [vp, i32, vp, vp]),
        "sfem_collocated_mass": (i32, [vp, vp]),
        "sfem_pcg": (i32, [vp, i32, i32, vp, vp, C.POINTER(PcgOpts), C.POINTER(PcgInfo)]),
        "sfem_grad_nu": (i32, [vp, i32, vp, vp, vp]),
        "sfem_get_info": (i32, [vp, C.POINTER(CtxInfo)]),
        "sfem_setup_pressure": (i32, [vp, vp, i64]),
        "sfem_stokes_apply": (i32, [vp, vp, vp, vp, vp]),
        "sfem_convection": (i32, [vp, vp, vp]),
        "sfem_weak_op": (i32, [vp, i32, vp, vp]),
        "sfem_lincomb": (i32, [vp, i32, C.POINTER(dbl), C.POINTER(vp), vp, vp, i64, i32, vp]),
        "sfem_bdf_ext_weights": (i32, [i32, C.POINTER(dbl), C.POINTER(dbl)]),
        "sfem_flow_create": (i32, [i32, vp, i32, i64, vp, vp, i64, vp, C.POINTER(FlowOpts), C.POINTER(vp)]),
        "sfem_flow_destroy": (None, [vp]),
        "sfem_flow_last_error": (C.c_char_p, [vp]),
        "sfem_flow_set_stream": (i32, [vp, vp]),
        "sfem_flow_step": (i32, [vp, vp, vp, vp, vp, C.POINTER(FlowInfo)]),
        "sfem_lor_setup": (i32, [vp, i32, C.POINTER(LorInfo)]),
        "sfem_lor_apply": (i32, [vp, i32, vp, vp]),
        "sfem_lor_vcycle": (i32, [vp, i32, i32, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
