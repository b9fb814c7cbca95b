"""ctypes loader for libac.so (argument marshalling only).

``import torch`` happens first so that libac binds to the HIP runtime torch
already loaded (both carry the soname libamdhip64.so.7): one runtime, one
device context, and torch's stream handles are valid inside libac.

The library must have been built (``paper_2105_09671_amd.build.build()``);
there is no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before libac)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libac.so")

AC_OK, AC_ERR_INVALID_ARG, AC_ERR_UNSTABLE, AC_ERR_UNSUPPORTED, AC_ERR_HIP, AC_ERR_NOMEM = range(6)
AC_F32, AC_F64 = 0, 1


class AcTune(ctypes.Structure):
    _fields_ = [("tb_depth", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("kernel", ctypes.c_int32)]


class AcPlan(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tb_depth", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("tile_z", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("launches", ctypes.c_int64), ("copy_back", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AcInstance2D(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("work", ctypes.c_void_p), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("h", ctypes.c_double), ("dt", ctypes.c_double),
                ("eps", ctypes.c_double)]


class AcInstance3D(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("work", ctypes.c_void_p), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("h", ctypes.c_double),
                ("dt", ctypes.c_double), ("eps", ctypes.c_double)]


class AcBatchInfo(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("items", ctypes.c_int32), ("tb_depth", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("copy_back", ctypes.c_int32), ("lds_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


AC_TUNE_2D, AC_TUNE_3D, AC_TUNE_BATCHED = 2, 3, 4

KERNEL_NAMES = {0: "tile2d_kernel (resident)", 1: "tile2d_kernel", 2: "stream3d_kernel",
                3: "tile2d_inplace_kernel", 4: "tile2d_reg_kernel", 5: "reg3d_kernel",
                6: "tile2d_regw_kernel"}


class AcError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__("%s failed: status %d (%s)" % (fn, status, msg))
        self.status = status


_lib = None

_vp, _i32, _i64, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double

SIGNATURES = {
    "ac_step_2d": ([_vp, _vp, _i32, _i32, _dbl, _dbl, _dbl, _i64, _i32, _vp], _i32),
    "ac_step_2d_tuned": ([_vp, _vp, _i32, _i32, _dbl, _dbl, _dbl, _i64, _i32,
                          ctypes.POINTER(AcTune), _vp], _i32),
    "ac_step_3d": ([_vp, _vp, _i32, _i32, _i32, _dbl, _dbl, _dbl, _i64, _i32, _vp], _i32),
    "ac_step_3d_tuned": ([_vp, _vp, _i32, _i32, _i32, _dbl, _dbl, _dbl, _i64, _i32,
                          ctypes.POINTER(AcTune), _vp], _i32),
    "ac_plan_2d": ([_i32, _i32, _i64, _i32, ctypes.POINTER(AcTune), ctypes.POINTER(AcPlan)], _i32),
    "ac_plan_3d": ([_i32, _i32, _i32, _i64, _i32, ctypes.POINTER(AcTune),
                    ctypes.POINTER(AcPlan)], _i32),
    "ac_step_batched": ([ctypes.POINTER(AcInstance2D), _i32, _i64, _i32, _vp], _i32),
    "ac_step_batched_tuned": ([ctypes.POINTER(AcInstance2D), _i32, _i64, _i32,
                               ctypes.POINTER(AcTune), ctypes.POINTER(AcBatchInfo), _vp], _i32),
    "ac_batched_set_persistent": ([_i32], None),
    "ac_step_batched_3d": ([ctypes.POINTER(AcInstance3D), _i32, _i64, _i32,
                            ctypes.POINTER(AcTune), ctypes.POINTER(AcBatchInfo), _vp], _i32),
    "ac_step_batched_masked": ([ctypes.POINTER(AcInstance2D), _i32, _i64, _i32,
                                ctypes.POINTER(AcTune), _vp, ctypes.POINTER(AcBatchInfo), _vp], _i32),
    "ac_batched_release": ([], _i32),
    "ac_batched_set_spin_limit": ([_i64], None),
    "ac_autotune_2d": ([_i32, _i32, _i32, _i64, ctypes.POINTER(AcTune), _vp], _i32),
    "ac_autotune_3d": ([_i32, _i32, _i32, _i32, _i64, ctypes.POINTER(AcTune), _vp], _i32),
    "ac_autotune_batched": ([ctypes.POINTER(AcInstance2D), _i32, _i32, _i64,
                             ctypes.POINTER(AcTune), _vp], _i32),
    "ac_autotune": ([_i32, _i32, ctypes.c_char_p], _i32),
    "ac_tune_save": ([ctypes.c_char_p], _i32),
    "ac_tune_load": ([ctypes.c_char_p], _i32),
    "ac_tune_clear": ([], None),
    "ac_tune_count": ([], _i32),
    "ac_sur_num_params": ([], _i64),
    "ac_sur_create": ([ctypes.POINTER(_vp), _i32, _i32, _vp], _i32),
    "ac_sur_destroy": ([_vp], None),
    "ac_sur_set_stream": ([_vp, _vp], _i32),
    "ac_sur_set_weights": ([_vp, ctypes.POINTER(ctypes.c_float), _i64], _i32),
    "ac_sur_get_weights": ([_vp, ctypes.POINTER(ctypes.c_float), _i64], _i32),
    "ac_sur_forward": ([_vp, _vp, _vp, _i32], _i32),
    "ac_sur_infer": ([_vp, _vp, _vp, _i32], _i32),
    "ac_sur_loss": ([_vp, _vp, _i32, _vp], _i32),
    "ac_sur_backward": ([_vp, _vp, _i32], _i32),
    "ac_sur_get_grads": ([_vp, ctypes.POINTER(ctypes.c_float), _i64], _i32),
    "ac_sur_adam_step": ([_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                          _i64], _i32),
    "ac_judge_2d": ([_vp, _vp, _i32, _i32, _i32, _dbl, _i32, _vp, _vp, _vp, _vp], _i32),
    "ac_err_2d": ([_vp, _vp, _vp, _vp, _i32, _i32, _dbl, _dbl, _dbl, _i64, _vp, _vp, _vp], _i32),
    "ac_err_3d": ([_vp, _vp, _vp, _vp, _i32, _i32, _i32, _dbl, _dbl, _dbl, _i64, _vp, _vp, _vp],
                  _i32),
    "ac_judge_workspace_bytes": ([_i32], _i64),
    "ac_judge_2d_noalloc": ([_vp, _vp, _i32, _i32, _i32, _dbl, _i32, _vp, _vp, _vp], _i32),
    "ac_check": ([_vp], _i32),
    "ac_status_string": ([_i32], ctypes.c_char_p),
    "ac_last_error": ([], ctypes.c_char_p),
    "ac_version": ([], _i32),
}


def lib():
    """The loaded libac (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libac.so is not built at %s; run __graft_entry__.build() "
                               "(there is no non-HIP fallback)" % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def check(status: int, fn: str) -> None:
    if status != AC_OK:
        msg = lib().ac_last_error().decode()
        raise AcError(status, fn, msg or lib().ac_status_string(status).decode())
