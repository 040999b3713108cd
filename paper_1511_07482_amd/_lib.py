"""ctypes view of libkdefft (include/kdefft.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library shares with torch)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkdefft.so")

OK = 0
FFT_SCHEDULES = 6
E_ARG, E_NOT_SPD, E_ODD_R, E_OUT_OF_GRID, E_OVERFLOW, E_WORKSPACE, E_HIP, E_UNSUPPORTED = range(-1, -9, -1)
OP_GRID_AUTO, OP_PSI_PLAIN, OP_PSI_FUSED, OP_PREPARE, OP_PSI_BATCH, OP_SCV_BATCH, OP_SCV_PLAIN, OP_AUTOTUNE, \
    OP_PSI_FFTL, OP_PREPARE_AUTO = range(1, 11)
PSI_PLAIN, PSI_FUSED = 0, 1
FUN_PSI, FUN_SCV_OBJ, FUN_SCV_OBJGRAD, FUN_SCV_GRAD, FUN_ETA1, FUN_ETA2 = range(6)
MAX_BATCH_DS = 64
MAX_PSI_DS = 32
MAX_TIMED = 4096
NOALLOC_BYTES = 16 << 20


class Grid(C.Structure):
    _fields_ = [("d", C.c_int32), ("M", C.c_int32 * 4), ("P", C.c_int32 * 4),
                ("lo", C.c_double * 4), ("delta", C.c_double * 4)]

    def to_dict(self):
        d = self.d
        import numpy as np
        return {"d": d, "M": np.array(self.M[:d], dtype=np.int64), "P": np.array(self.P[:d], dtype=np.int64),
                "lo": np.array(self.lo[:d]), "delta": np.array(self.delta[:d])}


class Dataset(C.Structure):
    _fields_ = [("grid", Grid), ("n", C.c_int64), ("G", C.c_double * 16),
                ("counts", C.c_void_p), ("spec", C.c_void_p), ("wmix", C.c_void_p), ("alag", C.c_void_p),
                ("scal", C.c_void_p), ("n_out", C.c_void_p), ("rec", C.c_void_p)]


EXPORTS = {
    "kdefft_strerror": (C.c_char_p, [C.c_int]),
    "kdefft_last_error_detail": (C.c_char_p, []),
    "kdefft_version": (C.c_int, []),
    "kdefft_unique_count": (C.c_int, [C.c_int, C.c_int]),
    "kdefft_unique_index": (C.c_int, [C.c_int, C.c_int, C.c_void_p]),
    "kdefft_grid_plan": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Grid)]),
    "kdefft_grid_auto": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                                   C.POINTER(Grid), C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_ws_bytes": (C.c_int, [C.POINTER(Grid), C.c_int, C.c_int, C.c_int64, C.POINTER(C.c_size_t)]),
    "kdefft_linbin": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p]),
    "kdefft_psi": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Grid), C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                             C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_check_binning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "kdefft_dataset_bytes": (C.c_int, [C.POINTER(Grid), C.POINTER(C.c_size_t)]),
    "kdefft_dataset_prepare": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Grid), C.c_void_p, C.c_void_p,
                                         C.c_size_t, C.POINTER(Dataset), C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_dataset_prepare_auto": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_double, C.c_void_p,
                                              C.c_void_p, C.c_size_t, C.POINTER(Dataset), C.c_void_p, C.c_size_t,
                                              C.c_void_p]),
    "kdefft_dataset_grid": (C.c_int, [C.POINTER(Dataset), C.POINTER(Grid), C.c_void_p]),
    "kdefft_psi_batch": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                   C.c_size_t, C.c_void_p]),
    "kdefft_scv_batch": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_scv_adjoint": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_scv_plain": (C.c_int, [C.POINTER(Dataset), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.c_void_p]),
    "kdefft_set_row_launch": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "kdefft_get_row_launch": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int),
                                        C.POINTER(C.c_int)]),
    "kdefft_lag_layout": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "kdefft_autotune": (C.c_int, [C.POINTER(Dataset), C.c_void_p, C.c_size_t, C.c_char_p, C.c_void_p]),
    "kdefft_crit_batch": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_crit_adjoint": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_pi_batch": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
    "kdefft_expand_full": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "kdefft_fftl_plan": (C.c_int, [C.POINTER(Grid), C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "kdefft_psi_fftl": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Grid), C.c_void_p, C.c_int, C.c_double,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_scv_batch_noalloc": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p]),
    "kdefft_minimize": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_minimize_ws_bytes": (C.c_int, [C.POINTER(Grid), C.c_int, C.c_int64, C.POINTER(C.c_size_t)]),
    "kdefft_set_fft_schedule": (C.c_int, [C.c_int, C.c_void_p, C.c_int]),
    "kdefft_get_fft_schedule": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_int)]),
    "kdefft_scv_walk_runs": (C.c_int, [C.POINTER(Dataset), C.c_int, C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_int64), C.c_void_p, C.c_size_t, C.c_void_p]),
    "kdefft_dataset_transform": (C.c_int, [C.POINTER(Dataset), C.c_void_p]),
    "kdefft_timing_start": (C.c_int, [C.c_int]),
    "kdefft_timing_stop": (C.c_int, [C.POINTER(C.c_float), C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int)]),
}

_lib = None


class KdefftError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        lib = load()
        name = lib.kdefft_strerror(code).decode()
        detail = lib.kdefft_last_error_detail().decode()
        super().__init__(f"{where}: {name} ({code}): {detail}")


def load():
    """Load libkdefft.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1511_07482_amd.build")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc, where):
    if rc != OK:
        raise KdefftError(rc, where)
