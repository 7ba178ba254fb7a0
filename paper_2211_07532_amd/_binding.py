"""ctypes view of libexpenc.so (the C ABI declared in include/expenc.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  Importing this module fails loudly if the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libexpenc.so")

EXPENC_OK = 0
EXPENC_EINVAL = -1
EXPENC_EWORKSPACE = -2
EXPENC_EHIP = -3
EXPENC_EUNSUPPORTED = -4
EXPENC_ENONFINITE = -5
EXPENC_EDIVERGED = -6
EXPENC_BATCH_FORKED = 0
EXPENC_BATCH_GROUPED = 1
EXPENC_ANCHOR_SPLIT, EXPENC_ANCHOR_FP32, EXPENC_ANCHOR_ENDS = 0, 1, 2

FP32, BF16_SPLIT, FP16_SPLIT = 0, 1, 2
HAAR, DB4 = 0, 1
BASIS_MAPS, BASIS_SH = 0, 1
WS_FORWARD, WS_ADJOINT, WS_FISTA, WS_LIPSCHITZ, WS_CG, WS_FIELD_GRAD = range(6)

_c_int = ctypes.c_int32
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class ExpencOp(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("ncoils", ctypes.c_int32), ("nbasis", ctypes.c_int32),
        ("nsamples", ctypes.c_int64),
        ("basis", _vp), ("coef", _vp), ("time", _vp), ("dw0", _vp), ("smaps", _vp),
        ("basis_kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("fov_x", ctypes.c_double), ("fov_y", ctypes.c_double), ("z0", ctypes.c_double),
    ]


class FistaOpts(ctypes.Structure):
    _fields_ = [
        ("n_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("wavelet", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("nx_pad", ctypes.c_int32), ("ny_pad", ctypes.c_int32),
        ("ista", ctypes.c_int32), ("refine_every", ctypes.c_int32),
        ("n_power", ctypes.c_int32), ("batch_launch", ctypes.c_int32),
        ("lipschitz", ctypes.c_double), ("lambda_", ctypes.c_double),
        ("lambda_factor", ctypes.c_double),
        ("power_v0", _vp), ("objective", _vp), ("scalars", _vp),
        ("anchor", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class BalancedOpts(ctypes.Structure):
    _fields_ = [
        ("n_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("wavelet", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("refine_every", ctypes.c_int32), ("n_power", ctypes.c_int32),
        ("ista", ctypes.c_int32), ("anchor", ctypes.c_int32),
        ("lipschitz", ctypes.c_double), ("kappa", ctypes.c_double), ("lambda_scale", ctypes.c_double),
        ("power_v0", _vp), ("lambda_", _vp), ("scalars", _vp),
    ]


# name -> (restype, argtypes); every symbol include/expenc.h declares
SIGNATURES = {
    "expenc_sh_basis": (ctypes.c_int, [_c_int, _c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       _c_int, _vp, _vp]),
    "expenc_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _c_int, _c_int, _c_int]),
    "expenc_forward": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "expenc_forward_static": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _vp, _vp, _vp]),
    "expenc_adjoint": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "expenc_lipschitz": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _vp, _vp, _vp, ctypes.c_size_t,
                                        _vp]),
    "wavelet_fwd": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp]),
    "wavelet_inv": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp]),
    "soft_threshold": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _vp, _vp, ctypes.c_float, _vp]),
    "wavelet_prox": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp, _vp, _vp,
                                    ctypes.c_double, _vp, _vp]),
    "fista_solve": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _vp, _vp, ctypes.POINTER(FistaOpts), _vp,
                                   ctypes.c_size_t, _vp]),
    "cg_solve": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _vp, _vp, ctypes.POINTER(FistaOpts), _vp,
                                ctypes.c_size_t, _vp]),
    "expenc_field_grad": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _vp, _vp, _vp, _vp, _vp,
                                         ctypes.c_size_t, _vp]),
    "soft_threshold_vjp": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp, ctypes.c_float, _vp]),
    "fista_batched_workspace_size": (ctypes.c_size_t, [_c_int, ctypes.POINTER(ExpencOp), _c_int,
                                                       ctypes.POINTER(FistaOpts)]),
    "fista_solve_batched": (ctypes.c_int, [_c_int, ctypes.POINTER(ExpencOp), _c_int, ctypes.POINTER(_vp),
                                           ctypes.POINTER(_vp), ctypes.POINTER(FistaOpts), _vp, ctypes.c_size_t,
                                           _vp]),
    "expenc_coil_workspace_size": (ctypes.c_size_t, [_c_int, ctypes.c_int64]),
    "expenc_prewhiten": (ctypes.c_int, [_c_int, _vp, ctypes.c_int64, _vp, _c_int, _vp, _vp, ctypes.c_size_t, _vp]),
    "expenc_coil_compress": (ctypes.c_int, [_c_int, _c_int, ctypes.c_int64, _vp, _c_int, _vp, _vp, _vp, _vp, _vp,
                                            _vp, ctypes.c_size_t, _vp]),
    "expenc_swt_workspace_size": (ctypes.c_size_t, [_c_int, _c_int, _c_int, _c_int]),
    "swt_fwd": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "swt_inv": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "expenc_sigma_workspace_size": (ctypes.c_size_t, [_c_int, _c_int, _c_int, _c_int]),
    "expenc_sigma_weights": (ctypes.c_int, [_c_int, _c_int, _c_int, _c_int, _vp, ctypes.c_double, _vp, _vp, _vp,
                                            ctypes.c_size_t, _vp]),
    "fista_balanced_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(ExpencOp), _c_int,
                                                        ctypes.POINTER(BalancedOpts)]),
    "fista_balanced_solve": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _vp, _vp, ctypes.POINTER(BalancedOpts),
                                            _vp, ctypes.c_size_t, _vp]),
    "expenc_set_tuning": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _c_int, _c_int]),
    "expenc_plan_info": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _c_int,
                                        ctypes.POINTER(ctypes.c_int64)]),
    "expenc_plan_info_ex": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _c_int,
                                           ctypes.POINTER(ctypes.c_int64), _c_int]),
    "expenc_set_launch_shape": (ctypes.c_int, [ctypes.POINTER(ExpencOp), _c_int, _c_int, _c_int, _c_int, _c_int]),
    "expenc_kernel_timing": (ctypes.c_int, [_c_int, ctypes.POINTER(ctypes.c_double)]),
    "expenc_solve_status": (ctypes.c_int, [_vp, _vp]),
    "expenc_axpby": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, _vp, ctypes.c_double, _vp, _vp, _vp]),
    "expenc_last_error": (ctypes.c_char_p, []),
}


class LibraryMissing(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded library (loads it on first use; raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise LibraryMissing(
                f"{_LIB_PATH} is missing: build it with paper_2211_07532_amd.build.build() "
                "(hipcc, gfx950). There is no fallback path.")
        h = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if not hasattr(h, name):
                continue
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def path() -> str:
    return _LIB_PATH


class ExpencError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().expenc_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != EXPENC_OK:
        raise ExpencError(status, where)
