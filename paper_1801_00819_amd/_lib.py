"""ctypes binding of libbrrlsm.so (the C ABI declared in include/brrlsm.h).

Argument marshalling only: every step of the computation runs in the HIP
library. Importing this module does not load the library; ``lib()`` does, and
raises if the library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbrrlsm.so")

BRLS_OK = 0
BRLS_EINVAL = -1
BRLS_ENOMEM = -2
BRLS_EFULL = -3
BRLS_ENOSHOT = -4
BRLS_EBREAKDOWN = -5
BRLS_ENONFINITE = -6
BRLS_EDEVICE = -7
BRLS_EDUP = -8

BRLS_DEVICE_PTRS = 1

BRLS_EXEC_PLAIN = 0
BRLS_EXEC_BATCHED = 1
BRLS_EXEC_GRAPH = 2
BRLS_EXEC_PERSISTENT = 3

ERROR_NAMES = {
    BRLS_EINVAL: "EINVAL", BRLS_ENOMEM: "ENOMEM", BRLS_EFULL: "EFULL",
    BRLS_ENOSHOT: "ENOSHOT", BRLS_EBREAKDOWN: "EBREAKDOWN",
    BRLS_ENONFINITE: "ENONFINITE", BRLS_EDEVICE: "EDEVICE", BRLS_EDUP: "EDUP",
}


class brls_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("nb", ctypes.c_int32), ("nt_max", ctypes.c_int32),
                ("nrec_max", ctypes.c_int32), ("q_max", ctypes.c_int32),
                ("h", ctypes.c_double), ("dt", ctypes.c_double),
                ("lambda_", ctypes.c_double),
                ("ckpt_interval", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class brls_shot(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("sz", ctypes.c_int32),
                ("sy", ctypes.c_int32), ("sx", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("nrec", ctypes.c_int32),
                ("f0", ctypes.c_double),
                ("rec", ctypes.POINTER(ctypes.c_int32)),
                ("data", ctypes.c_void_p)]


class brls_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("s0_norm", ctypes.c_double),
                ("s_norm", ctypes.c_double), ("r_norm", ctypes.c_double),
                ("seconds", ctypes.c_double), ("ref_norm", ctypes.c_double)]


class brls_kstat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class brls_ssf_grid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dz", ctypes.c_double),
                ("nt", ctypes.c_int32), ("dt", ctypes.c_double),
                ("fmin", ctypes.c_double), ("fmax", ctypes.c_double),
                ("ntap", ctypes.c_int32), ("nrec_max", ctypes.c_int32),
                ("q_max", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


class brls_ssf_shot(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("xs", ctypes.c_int32),
                ("nrec", ctypes.c_int32), ("f0", ctypes.c_double),
                ("rec", ctypes.POINTER(ctypes.c_int32)),
                ("data", ctypes.c_void_p)]


# (name, restype, argtypes) of every exported symbol
_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
SIGNATURES = [
    ("brls_open", _I32, [ctypes.POINTER(brls_grid), _VP, _VP,
                         ctypes.POINTER(_VP)]),
    ("brls_close", None, [_VP]),
    ("brls_last_error", ctypes.c_char_p, [_VP]),
    ("brls_update", _I32, [_VP, ctypes.POINTER(brls_shot)]),
    ("brls_downdate", _I32, [_VP, _I64]),
    ("brls_set_data", _I32, [_VP, _I64, _VP]),
    ("brls_window", _I32, [_VP, ctypes.POINTER(_I64), _I32,
                           ctypes.POINTER(_I32)]),
    ("brls_window_data_size", _I32, [_VP, ctypes.POINTER(_I64)]),
    ("brls_solve_window", _I32, [_VP, _I32, ctypes.c_double,
                                 ctypes.POINTER(brls_stats)]),
    ("brls_solve_history", _I32, [_VP, _I32, _VP, _VP, _VP,
                                  ctypes.POINTER(_I32)]),
    ("brls_set_chains", _I32, [_VP, _I32]),
    ("brls_get_chains", _I32, [_VP, ctypes.POINTER(_I32)]),
    ("brls_image", _I32, [_VP, _VP]),
    ("brls_set_image", _I32, [_VP, _VP]),
    ("brls_image64", _I32, [_VP, _VP]),
    ("brls_set_image64", _I32, [_VP, _VP]),
    ("brls_set_precond", _I32, [_VP, _I32]),
    ("brls_set_regularization", _I32, [_VP, _I32]),
    ("brls_set_precision", _I32, [_VP, _I32, _I32]),
    ("brls_get_precision", _I32, [_VP, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)]),
    ("brls_set_shot_weight", _I32, [_VP, ctypes.c_int64, ctypes.c_double]),
    ("brls_get_shot_weight", _I32,
     [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    ("brls_get_regularization", _I32, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    ("brls_get_precond", _I32, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    ("brls_illumination", _I32, [_VP, _VP]),
    ("brls_apply_born", _I32, [_VP, _VP, _VP]),
    ("brls_apply_adjoint", _I32, [_VP, _VP, _VP]),
    ("brls_apply_adjoint_static", _I32, [_VP, _VP, _VP]),
    ("brls_background_window", _I32, [_VP, _VP]),
    ("brls_set_exec", _I32, [_VP, _I32]),
    ("brls_set_spin_limit", _I32, [_VP, _I32]),
    ("brls_set_zchunk", _I32, [_VP, _I32]),
    ("brls_get_zchunk", _I32, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    ("brls_set_tile", _I32, [_VP, _I32]),
    ("brls_tile_count", _I32, [ctypes.POINTER(_I32)]),
    ("brls_tile_info", _I32, [_I32, ctypes.POINTER(_I32),
                              ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                              ctypes.POINTER(_I32)]),
    ("brls_tile3_count", _I32, [ctypes.POINTER(_I32)]),
    ("brls_tile3_info", _I32, [_I32, ctypes.POINTER(_I32),
                               ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("brls_set_shots_per_block", _I32, [_VP, _I32]),
    ("brls_get_tile", _I32, [_VP, ctypes.POINTER(_I32),
                             ctypes.POINTER(_I32)]),
    ("brls_set_resident_grid", _I32, [_VP, _I32]),
    ("brls_get_resident_grid", _I32, [_VP, ctypes.POINTER(_I32)]),
    ("brls_set_tuning", _I32, [_VP, _I32, _I32, _I32, _I32, _I32]),
    ("brls_get_tuning", _I32, [_VP] + [ctypes.POINTER(_I32)] * 5),
    ("brls_autotune", _I32, [_VP, ctypes.POINTER(_I32)]),
    ("brls_kernel_timing", _I32, [_VP, _I32]),
    ("brls_kernel_stats", _I32, [_VP, ctypes.POINTER(brls_kstat), _I32,
                                 ctypes.POINTER(_I32)]),
    ("brls_memory_bytes", _I32, [_VP, ctypes.POINTER(_I64)]),
    ("brls_sync", _I32, [_VP]),
    # split-step Fourier context (include/brrlsm_ssf.h)
    ("brls_ssf_open", _I32, [ctypes.POINTER(brls_ssf_grid), _VP, _VP,
                             ctypes.POINTER(_VP)]),
    ("brls_ssf_close", None, [_VP]),
    ("brls_ssf_last_error", ctypes.c_char_p, [_VP]),
    ("brls_ssf_band", _I32, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                             ctypes.POINTER(ctypes.c_double)]),
    ("brls_ssf_update", _I32, [_VP, ctypes.POINTER(brls_ssf_shot)]),
    ("brls_ssf_downdate", _I32, [_VP, _I64]),
    ("brls_ssf_window", _I32, [_VP, ctypes.POINTER(_I64), _I32,
                               ctypes.POINTER(_I32)]),
    ("brls_ssf_window_data_size", _I32, [_VP, ctypes.POINTER(_I64)]),
    ("brls_ssf_apply_born", _I32, [_VP, _VP, _VP]),
    ("brls_ssf_apply_adjoint", _I32, [_VP, _VP, _VP]),
    ("brls_ssf_observed", _I32, [_VP, _VP]),
    ("brls_ssf_solve_window", _I32, [_VP, _I32, ctypes.c_double,
                                     ctypes.POINTER(brls_stats)]),
    ("brls_ssf_set_precond", _I32, [_VP, _I32]),
    ("brls_ssf_get_precond", _I32, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    ("brls_ssf_illumination", _I32, [_VP, _VP]),
    ("brls_ssf_set_regularization", _I32, [_VP, _I32]),
    ("brls_ssf_set_shot_weight", _I32, [_VP, ctypes.c_int64, ctypes.c_double]),
    ("brls_ssf_get_shot_weight", _I32,
     [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    ("brls_ssf_get_regularization", _I32,
     [_VP, ctypes.POINTER(ctypes.c_int32)]),
    ("brls_ssf_image", _I32, [_VP, _VP]),
    ("brls_ssf_set_image", _I32, [_VP, _VP]),
    ("brls_ssf_kernel_timing", _I32, [_VP, _I32]),
    ("brls_ssf_kernel_stats", _I32, [_VP, ctypes.POINTER(brls_kstat), _I32,
                                     ctypes.POINTER(_I32)]),
    ("brls_ssf_memory_bytes", _I32, [_VP, ctypes.POINTER(_I64)]),
    ("brls_ssf_sync", _I32, [_VP]),
]

_lib = None


def lib(path: str = LIB_PATH):
    """Load libbrrlsm.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        # Load torch's HIP runtime first when torch is installed, so the
        # library binds to the same runtime instance (one per process): the
        # device pointers and streams torch hands over are only valid there.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(path):
            raise ImportError(
                f"{path} is not built; run __graft_entry__.build() or "
                "python paper_1801_00819_amd/build.py")
        L = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class BrlsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc: int, ctx=None):
    if rc != BRLS_OK:
        msg = lib().brls_last_error(ctx)
        raise BrlsError(rc, msg.decode() if msg else "")
    return rc


def check_ssf(rc: int, ctx=None):
    if rc != BRLS_OK:
        msg = lib().brls_ssf_last_error(ctx)
        raise BrlsError(rc, msg.decode() if msg else "")
    return rc
