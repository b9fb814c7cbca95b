"""Python API over libac: device tensors in, the C ABI does all stepping.

torch supplies device memory and the current stream; every step runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_work_cache: dict = {}


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return L.AC_F32
    if t.dtype == torch.float64:
        return L.AC_F64
    raise TypeError("phi must be float32 or float64, got %s" % t.dtype)


def _check_tensor(phi: torch.Tensor, ndim: int) -> None:
    if not isinstance(phi, torch.Tensor) or not phi.is_cuda:
        raise TypeError("phi must be a device tensor")
    if phi.dim() != ndim:
        raise ValueError("phi must have %d dimensions, got %d" % (ndim, phi.dim()))
    if not phi.is_contiguous():
        raise ValueError("phi must be contiguous")


def work_like(phi: torch.Tensor) -> torch.Tensor:
    """A cached scratch buffer of phi's size, dtype and device."""
    key = (phi.device, phi.dtype, phi.numel())
    w = _work_cache.get(key)
    if w is None:
        w = torch.empty(phi.numel(), dtype=phi.dtype, device=phi.device)
        _work_cache[key] = w
    return w


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _tune(tune):
    if tune is None:
        return None
    if isinstance(tune, L.AcTune):
        return ctypes.byref(tune)
    t = L.AcTune(int(tune.get("tb_depth", 0)), int(tune.get("tile_x", 0)),
                 int(tune.get("tile_y", 0)), int(tune.get("tile_z", 0)))
    return ctypes.byref(t)


def step2d(phi: torch.Tensor, h: float, dt: float, eps: float, nsteps: int,
           work: torch.Tensor | None = None, tune=None, stream=None) -> torch.Tensor:
    """Advance phi (shape (ny, nx)) in place by nsteps explicit steps."""
    _check_tensor(phi, 2)
    ny, nx = phi.shape
    w = work if work is not None else work_like(phi)
    st = L.lib().ac_step_2d_tuned(phi.data_ptr(), w.data_ptr(), nx, ny, float(h), float(dt),
                                  float(eps), int(nsteps), _dtype_code(phi), _tune(tune),
                                  _stream(stream))
    L.check(st, "ac_step_2d")
    return phi


def step3d(phi: torch.Tensor, h: float, dt: float, eps: float, nsteps: int,
           work: torch.Tensor | None = None, tune=None, stream=None) -> torch.Tensor:
    """Advance phi (shape (nz, ny, nx)) in place by nsteps explicit steps."""
    _check_tensor(phi, 3)
    nz, ny, nx = phi.shape
    w = work if work is not None else work_like(phi)
    st = L.lib().ac_step_3d_tuned(phi.data_ptr(), w.data_ptr(), nx, ny, nz, float(h), float(dt),
                                  float(eps), int(nsteps), _dtype_code(phi), _tune(tune),
                                  _stream(stream))
    L.check(st, "ac_step_3d")
    return phi


def check(stream=None) -> None:
    """Synchronise the stream and raise on a pending HIP error."""
    L.check(L.lib().ac_check(_stream(stream)), "ac_check")


def plan2d(nx: int, ny: int, nsteps: int, dtype=torch.float32, tune=None) -> dict:
    """The launch plan ac_step_2d would use (kernel, depth, tile, launches)."""
    p = L.AcPlan()
    code = L.AC_F64 if dtype == torch.float64 else L.AC_F32
    L.check(L.lib().ac_plan_2d(nx, ny, int(nsteps), code, _tune(tune), ctypes.byref(p)), "ac_plan_2d")
    return p.as_dict()


def plan3d(nx: int, ny: int, nz: int, nsteps: int, dtype=torch.float32, tune=None) -> dict:
    p = L.AcPlan()
    code = L.AC_F64 if dtype == torch.float64 else L.AC_F32
    L.check(L.lib().ac_plan_3d(nx, ny, nz, int(nsteps), code, _tune(tune), ctypes.byref(p)),
            "ac_plan_3d")
    return p.as_dict()
