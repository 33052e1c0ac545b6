"""ctypes binding of libstpi.so (argument marshalling only).

The library is the only compute path: if it is missing this module raises at
import time instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstpi.so")

STPI_OK = 0
STPI_EINVAL = 1
STPI_EUNSUPPORTED = 2
STPI_EZERO_NORM = 3
STPI_ENONFINITE = 4
STPI_EHIP = 5
STPI_EWORKSPACE = 6

STPI_F32 = 0
STPI_BF16 = 1
STPI_F64 = 2
STPI_MAX_RS = 16
STPI_MAX_RT = 8


class Problem(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("sigma_s", ctypes.c_float), ("sigma_t", ctypes.c_float),
                ("r_s", ctypes.c_int32), ("r_t", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class Clip(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("T", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("residual", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("rayleigh", ctypes.c_double), ("first_residuals", ctypes.c_double * 2)]

    def as_dict(self):
        return dict(iters=self.iters, converged=bool(self.converged), flags=self.flags, status=self.status,
                    residual=self.residual, lambda_=self.lambda_, rayleigh=self.rayleigh,
                    r1=self.first_residuals[0], r2=self.first_residuals[1])


# (name, restype, argtypes); pointers to device memory and streams are void*.
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_PP = ctypes.POINTER(Problem)
_RP = ctypes.POINTER(Result)
PROTOTYPES = [
    ("stpi_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("stpi_last_error", ctypes.c_char_p, []),
    ("stpi_version", ctypes.c_char_p, []),
    ("stpi_workspace_bytes", _sz, [_PP]),
    ("stpi_step", ctypes.c_int, [_PP, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_step_noalloc_scratch_bytes", _sz, [_PP]),
    ("stpi_step_noalloc", ctypes.c_int, [_PP, _vp, _vp, ctypes.c_double, _vp, _vp, _vp]),
    ("stpi_iterate", ctypes.c_int, [_PP, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp, _sz, _RP, _vp]),
    ("stpi_sfseg_unary", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _vp, ctypes.c_double, _vp, _vp]),
    ("stpi_sfseg_workspace_bytes", _sz, [_PP]),
    ("stpi_sfseg_step", ctypes.c_int, [_PP, _vp, _vp, ctypes.c_double, _vp, ctypes.c_double, _vp, _vp, _vp, _sz,
                                       _vp]),
    ("stpi_sfseg_iterate", ctypes.c_int, [_PP, _vp, _vp, ctypes.c_double, _vp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, _vp, _sz, _RP, _vp]),
    ("stpi_window_start", ctypes.c_int, [_PP, _vp, ctypes.c_int, _vp, _vp]),
    ("stpi_exp_workspace_bytes", _sz, [_PP]),
    ("stpi_exp_step", ctypes.c_int, [_PP, _vp, _vp, ctypes.c_double, _vp, ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_exp_iterate", ctypes.c_int, [_PP, _vp, _vp, ctypes.c_double, _vp, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, _vp, _sz, _RP, _vp]),
    ("stpi_combine_sigmoid_fwd", ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp,
                                                 _vp]),
    ("stpi_combine_sigmoid_bwd", ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp, _vp,
                                                 _sz, _vp]),
    ("stpi_softbin_fwd", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _vp, _vp, ctypes.c_double, ctypes.c_double,
                                        _vp, _vp, _vp, _sz, _vp]),
    ("stpi_softbin_bwd", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_focal_dice_workspace_bytes", _sz, [ctypes.c_int]),
    ("stpi_focal_dice", ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp, _vp, ctypes.c_double,
                                       ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_variant_count", ctypes.c_int, [ctypes.c_int]),
    ("stpi_variant_info", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]),
    ("stpi_launch_shape", ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]),
    ("stpi_downsample", ctypes.c_int, [ctypes.c_int] * 6 + [_vp, _vp, _vp]),
    ("stpi_upsample", ctypes.c_int, [ctypes.c_int] * 7 + [_vp, _vp, _vp, _vp]),
    ("stpi_coarse_problem", ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(Problem)]),
    ("stpi_scale", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _vp, ctypes.c_double, _vp, _vp, _vp]),
    ("stpi_set_variant", ctypes.c_int, [ctypes.c_int]),
    ("stpi_time_step", ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _sz, ctypes.c_int, ctypes.c_int, _vp,
                                      ctypes.POINTER(ctypes.c_double)]),
    ("stpi_time_chain_step", ctypes.c_int, [_PP, _vp, _vp, _vp, _sz, ctypes.c_int, ctypes.c_int, _vp,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    ("stpi_batch_plan", ctypes.c_int, [ctypes.POINTER(Clip), ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("stpi_batch_workspace_bytes", _sz, [_vp]),
    ("stpi_batch_info", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    ("stpi_batch_iterate", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp, _sz,
                                          _RP, _vp]),
    ("stpi_plan_destroy", None, [_vp]),
    ("stpi_autotune", ctypes.c_int, [_PP, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_double)]),
    ("stpi_autotune_load", ctypes.c_int, [ctypes.c_char_p]),
    ("stpi_autotune_clear", None, []),
    ("stpi_net_param_count", ctypes.c_int, []),
    ("stpi_net_prep_bytes", _sz, []),
    ("stpi_net_workspace_bytes", _sz, [_PP]),
    ("stpi_net_prepare", ctypes.c_int, [_vp, _vp, _vp]),
    ("stpi_net_forward", ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_net_backward", ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_net_warm_start", ctypes.c_int, [ctypes.c_int64, _vp, ctypes.c_float, _vp, _vp]),
    ("stpi_train_init", ctypes.c_int, [_PP, _vp, _vp, _vp]),
    ("stpi_train_step", ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_adjoint_step", ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_normalize", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp]),
    ("stpi_dot", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_combine_fwd", ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp]),
    ("stpi_combine_bwd", ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _sz,
                                        _vp]),
    ("stpi_bce", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("stpi_adamw", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, _vp]),
]

AUX_WS_BYTES = 512 * 1024
MAX_CHANNELS = 64
STPI_NOALLOC_SCRATCH_BYTES = 1 << 20


class StpiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"stpi error {status}: {message}")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libstpi.so not found at {path}: build it with "
                          f"`python -c 'import __graft_entry__ as g; g.build()'` or paper_2212_08058_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, res, args in PROTOTYPES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


def check(status: int) -> None:
    if status != STPI_OK:
        msg = lib.stpi_last_error().decode() or lib.stpi_status_string(status).decode()
        raise StpiError(status, msg)
