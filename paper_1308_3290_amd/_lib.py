"""ctypes view of libcgp.so: the C ABI of include/cgp.h, names unchanged.

Argument marshalling only; every step of the method runs in the library's
gfx950 kernels.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcgp.so")
# the measurement build (phase stamps; cgp_phase_stamps): a program that wants
# it sets LIB_PATH to this path before the first load()
STAMPS_LIB_PATH = os.path.join(_PKG, "libcgp_stamps.so")

CGP_OK, CGP_ERR_INVALID, CGP_ERR_UNSUPPORTED, CGP_ERR_DEVICE, CGP_ERR_NONFINITE = range(5)
CGP_F32, CGP_F64 = 0, 1
STATUS_NAMES = {0: "CGP_OK", 1: "CGP_ERR_INVALID", 2: "CGP_ERR_UNSUPPORTED",
                3: "CGP_ERR_DEVICE", 4: "CGP_ERR_NONFINITE"}


class cgp_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("level", ctypes.c_int32),
                ("nlayers", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("y0", ctypes.c_double), ("inv_re", ctypes.c_double),
                ("inv_ro", ctypes.c_double), ("f1", ctypes.c_double), ("f2", ctypes.c_double),
                ("drag", ctypes.c_double), ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
                ("solver", ctypes.c_int32), ("mg_cycles", ctypes.c_int32),
                ("fused_rows", ctypes.c_int32)]


class cgp_launch(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("b_tile", ctypes.c_int32), ("f_tile", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32)]


class CGPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_P = ctypes.c_void_p
_SZ = ctypes.c_size_t
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_CFG = ctypes.POINTER(cgp_config)

# name -> (restype, argtypes); every function of include/cgp.h
SIGNATURES = {
    "cgp_workspace_size": (_I32, [_CFG, ctypes.POINTER(_SZ)]),
    "cgp_create": (_I32, [_CFG, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "cgp_destroy": (_I32, [_P]),
    "cgp_step": (_I32, [_P, _P, _P, _P, _I32, _P]),
    "cgp_step_noalloc": (_I32, [_CFG, _P, _P, _P, _I32, _P]),
    "cgp_solve": (_I32, [_P, _P, _P, _P]),
    "cgp_time_state": (_I32, [_P, _P, _P]),
    "cgp_accumulate": (_I32, [_P, _P, _P, ctypes.c_double, _I32, _P]),
    "cgp_step_mean": (_I32, [_P, _P, _P, _I32, _P, _I32, _P]),
    "cgp_diagnostics": (_I32, [_P, _P, _P, _P, _P]),
    "cgp_check_finite": (_I32, [_P, _P, _I64, _P, _P]),
    "cgp_assert_finite": (_I32, [_P, _P, _I64, _P]),
    "cgp_tape_size": (_I32, [_CFG, _I32, ctypes.POINTER(_SZ)]),
    "cgp_adjoint_step": (_I32, [_P, _P, _P, _I32, _P, _P, _P, _SZ, _P]),
    "cgp_ensemble_offsets": (_I32, [_CFG, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "cgp_ensemble_workspace_size": (_I32, [_CFG, _I32, ctypes.POINTER(_SZ)]),
    "cgp_ensemble_create": (_I32, [_CFG, _I32, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "cgp_ensemble_step": (_I32, [_P, _P, _P, _I32, _I32, _P]),
    "cgp_time_passes": (_I32, [_P, _P, _P, _I32, ctypes.POINTER(ctypes.c_double), _P]),
    "cgp_time_step_passes": (_I32, [_P, _P, _P, _I32, ctypes.POINTER(ctypes.c_double), _P]),
    "cgp_set_launch": (_I32, [_P, ctypes.POINTER(cgp_launch), _P]),
    "cgp_get_launch": (_I32, [_P, ctypes.POINTER(cgp_launch), ctypes.POINTER(_I32)]),
    "cgp_persistent_fault": (_I32, [_P, ctypes.POINTER(_I32), _P]),
    "cgp_last_error": (ctypes.c_char_p, []),
    "cgp_version": (ctypes.c_char_p, []),
}

# Functions only the measurement build exports.
OPTIONAL_SIGNATURES = {
    "cgp_phase_stamps": (_I32, [_I32, ctypes.POINTER(ctypes.c_uint64), _I32,
                                ctypes.POINTER(_I32)]),
}

_lib = None


def load():
    """Load libcgp.so (or the library LIB_PATH names) once.  torch is imported
    first so that the library binds to the same HIP runtime instance torch
    uses (streams and pointers are shared)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1308_3290_amd.build` (there is no fallback path)")
    import torch  # noqa: F401  (HIP runtime first)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    for name, (res, args) in OPTIONAL_SIGNATURES.items():
        if hasattr(lib, name):
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != CGP_OK:
        msg = load().cgp_last_error().decode(errors="replace")
        raise CGPError(status, msg)


def call(name, *args):
    """Call a status-returning C function and raise CGPError on failure."""
    check(getattr(load(), name)(*args))
