"""ctypes binding of the C ABI declared in include/fvm.h.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libfvm.so``. Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfvm.so")

FVM_OK, FVM_EINVAL, FVM_EDEVICE, FVM_ECFL, FVM_ENONFINITE, FVM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FVM_EIO = -6
FVM_CLOSURE_LOGNORMAL, FVM_CLOSURE_MAXENT = 0, 1
FVM_ADV, FVM_EULER, FVM_SPRAY = 0, 1, 2
FVM_PERIODIC, FVM_TRANSMISSIVE, FVM_DIRICHLET = 0, 1, 2
FVM_LAYOUT_PLANES, FVM_LAYOUT_ROWS = 0, 1


class FvmError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _strerror(code)
        super().__init__(f"{what}: {msg} (status {code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("model", C.c_int), ("bc", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("npart_x", C.c_int), ("npart_y", C.c_int), ("ld", C.c_int), ("layout", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double), ("gamma", C.c_double),
        ("ax", C.c_double), ("ay", C.c_double), ("K", C.c_double),
        ("theta", C.c_double), ("s_eps", C.c_double), ("cfl", C.c_double),
        ("dt_max", C.c_double), ("closure", C.c_int),
    ]


_D = C.POINTER(C.c_double)
_V = C.c_void_p
_P = C.POINTER(Params)

# name -> (restype, argtypes); the same names as include/fvm.h
SIGNATURES = {
    "fvm_strerror": (C.c_char_p, [C.c_int]),
    "fvm_nvar": (C.c_int, [C.c_int]),
    "fvm_validate": (C.c_int, [_P]),
    "fvm_scratch_bytes": (C.c_size_t, [_P]),
    "fvm_create": (C.c_int, [_P, C.POINTER(_V)]),
    "fvm_destroy": (C.c_int, [_V]),
    "fvm_bind": (C.c_int, [_V, _V, _V, _V, _V, _V]),
    "fvm_set_stream": (C.c_int, [_V, _V]),
    "fvm_current": (C.c_int, [_V, C.POINTER(_V)]),
    "fvm_set_state": (C.c_int, [_V, _V, C.c_int]),
    "fvm_get_state": (C.c_int, [_V, _V, C.c_int]),
    "fvm_cfl_dt": (C.c_int, [_V, _V]),
    "fvm_cfl_dt_host": (C.c_int, [_V, _D, _D, _D]),
    "fvm_step": (C.c_int, [_V, C.c_double]),
    "fvm_run": (C.c_int, [_V, C.c_int, _V]),
    "fvm_run_dts": (C.c_int, [_V, C.c_int, _V]),
    "fvm_run_fixed": (C.c_int, [_V, C.c_int, C.c_double]),
    "fvm_set_boundary_states": (C.c_int, [_V, _V]),
    "fvm_set_adjoint_tiling": (C.c_int, [_V, C.c_int, C.c_int, C.c_int]),
    "fvm_set_halo_rows": (C.c_int, [_V, _V, _V]),
    "fvm_batch_set_schedule": (C.c_int, [_V, C.c_int, C.c_int]),
    "fvm_batch_set_layout": (C.c_int, [_V, C.c_int]),
    "fvm_set_resident_runs": (C.c_int, [_V, C.c_int]),
    "fvm_run_ckpt": (C.c_int, [_V, C.c_int, C.c_int, C.POINTER(_V), _V]),
    "fvm_run_noalloc": (C.c_int, [_P, _V, _V, _V, C.c_int, _V, _V, _V]),
    "fvm_sync": (C.c_int, [_V]),
    "fvm_get_status": (C.c_int, [_V, C.c_int]),
    "fvm_adjoint_run": (C.c_int, [_V, C.POINTER(_V), C.c_int, _V, C.c_int, _V, _V, _V]),
    "fvm_adjoint_step": (C.c_int, [_V, _V, C.c_double, _V, _V]),
    "fvm_set_tiling": (C.c_int, [_V, C.c_int, C.c_int]),
    "fvm_get_tiling": (C.c_int, [_V, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "fvm_set_cells_per_lane": (C.c_int, [_V, C.c_int]),
    "fvm_get_cells_per_lane": (C.c_int, [_V]),
    "fvm_autotune": (C.c_int, [_V, C.c_char_p]),
    "fvm_batch_create": (C.c_int, [C.c_int, _P, C.POINTER(C.c_size_t), C.POINTER(_V)]),
    "fvm_batch_destroy": (C.c_int, [_V]),
    "fvm_batch_scratch_bytes": (C.c_size_t, [_V]),
    "fvm_batch_bind": (C.c_int, [_V, _V, _V, _V, _V]),
    "fvm_batch_cfl": (C.c_int, [_V]),
    "fvm_batch_run": (C.c_int, [_V, C.c_int, _V]),
    "fvm_batch_run_per_grid": (C.c_int, [_V, C.c_int, _V]),
    "fvm_batch_current": (C.c_int, [_V, C.POINTER(_V)]),
    "fvm_batch_sync": (C.c_int, [_V]),
    "fvm_batch_set_tiling": (C.c_int, [_V, C.c_int, C.c_int]),
    "fvm_batch_autotune": (C.c_int, [_V, C.c_char_p]),
    "fvm_set_closure_buffer": (C.c_int, [_V, _V]),
    "fvm_autotune_adjoint": (C.c_int, [_V, _V, _V, _V, C.c_char_p]),
    "fvm_output_create": (C.c_int, [_V, _V, _V, _V, C.POINTER(_V)]),
    "fvm_output_snapshot": (C.c_int, [_V, C.c_char_p, C.c_longlong, C.c_double]),
    "fvm_output_wait": (C.c_int, [_V]),
    "fvm_output_destroy": (C.c_int, [_V]),
}

_lib = None


def lib():
    """The loaded library; raises if libfvm.so is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_1701_05431_amd.build` "
                "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().fvm_strerror(int(code)).decode()
    except Exception:  # library unavailable while formatting an error
        return "error"


def check(code: int, what: str) -> int:
    if code != FVM_OK:
        raise FvmError(code, what)
    return code
