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


def release_work() -> None:
    """Drop the cached scratch buffers (they are re-created on demand)."""
    _work_cache.clear()


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _tune(tune):
    if tune is None:
        return None
    if isinstance(tune, L.AcTune):
        return ctypes.byref(tune)
    t = L.AcTune(int(tune.get("tb_depth", 0)), int(tune.get("tile_x", 0)),
                 int(tune.get("tile_y", 0)), int(tune.get("tile_z", 0)), int(tune.get("kernel", 0)))
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


# ---------------------------------------------------------------- batched ----
class Batch:
    """Independent 2D grids packed into one phi buffer and one work buffer.

    ``fields`` are (ny, nx) arrays; ``params`` are (h, dt, eps) per grid.  Each
    grid starts on a 256-byte boundary.  ``views()`` returns the per-grid phi
    tensors (views into the packed buffer)."""

    def __init__(self, fields, params, dtype=torch.float32, device="cuda"):
        import numpy as np
        self.dtype = dtype
        elem = torch.tensor([], dtype=dtype).element_size()
        align = 256 // elem
        self.shapes = [tuple(np.shape(f)) for f in fields]
        self.offsets = []
        off = 0
        for (ny, nx) in self.shapes:
            self.offsets.append(off)
            off += (ny * nx + align - 1) // align * align
        self.total = off
        host = torch.zeros(off, dtype=dtype)
        for f, o, (ny, nx) in zip(fields, self.offsets, self.shapes):
            host[o:o + ny * nx] = torch.as_tensor(np.ascontiguousarray(f).ravel(), dtype=dtype)
        self.phi = host.to(device)
        self.work = torch.empty_like(self.phi)
        self.params = [tuple(float(v) for v in p) for p in params]
        self._arr = self._instances(self.phi, self.work)

    def _instances(self, phi, work):
        elem = phi.element_size()
        arr = (L.AcInstance2D * len(self.shapes))()
        for i, ((ny, nx), o, (h, dt, eps)) in enumerate(zip(self.shapes, self.offsets, self.params)):
            arr[i] = L.AcInstance2D(phi.data_ptr() + o * elem, work.data_ptr() + o * elem,
                                    nx, ny, h, dt, eps)
        return arr

    @property
    def cells(self) -> int:
        return sum(nx * ny for (ny, nx) in self.shapes)

    def views(self):
        return [self.phi[o:o + ny * nx].view(ny, nx) for o, (ny, nx) in zip(self.offsets, self.shapes)]

    def step(self, nsteps: int, tune=None, stream=None) -> dict:
        info = L.AcBatchInfo()
        st = L.lib().ac_step_batched_tuned(self._arr, len(self.shapes), int(nsteps),
                                           _dtype_code(self.phi), _tune(tune), ctypes.byref(info),
                                           _stream(stream))
        L.check(st, "ac_step_batched")
        return info.as_dict()

    def step_masked(self, nsteps: int, active: torch.Tensor, tune=None, stream=None) -> dict:
        """Step only the grids i with active[i] != 0 (int32 device tensor)."""
        if active.dtype != torch.int32 or not active.is_cuda or active.numel() != len(self.shapes):
            raise ValueError("int32 device tensor with one entry per grid expected")
        info = L.AcBatchInfo()
        st = L.lib().ac_step_batched_masked(self._arr, len(self.shapes), int(nsteps),
                                            _dtype_code(self.phi), _tune(tune), active.data_ptr(),
                                            ctypes.byref(info), _stream(stream))
        L.check(st, "ac_step_batched_masked")
        return info.as_dict()

    def autotune(self, probe_steps: int = 200, stream=None) -> dict:
        best = L.AcTune()
        L.check(L.lib().ac_autotune_batched(self._arr, len(self.shapes), _dtype_code(self.phi),
                                            int(probe_steps), ctypes.byref(best), _stream(stream)),
                "ac_autotune_batched")
        return {k: getattr(best, k) for k, _ in best._fields_}


def batched_persistent(on: bool) -> None:
    """Choose how batched calls execute: one persistent launch with a phase
    barrier (True) or a captured graph of one launch per phase (False, the
    default).  Results are bitwise the same."""
    L.lib().ac_batched_set_persistent(1 if on else 0)


class Batch3D:
    """Independent 3D grids packed into one phi and one work buffer; ``fields``
    are (nz, ny, nx) arrays, ``params`` (h, dt, eps) per grid."""

    def __init__(self, fields, params, dtype=torch.float32, device="cuda"):
        import numpy as np
        self.dtype = dtype
        align = 256 // torch.tensor([], dtype=dtype).element_size()
        self.shapes = [tuple(np.shape(f)) for f in fields]
        self.offsets, off = [], 0
        for sh in self.shapes:
            self.offsets.append(off)
            off += (int(np.prod(sh)) + align - 1) // align * align
        host = torch.zeros(off, dtype=dtype)
        for f, o, sh in zip(fields, self.offsets, self.shapes):
            n = int(np.prod(sh))
            host[o:o + n] = torch.as_tensor(np.ascontiguousarray(f).ravel(), dtype=dtype)
        self.phi = host.to(device)
        self.work = torch.empty_like(self.phi)
        self.params = [tuple(float(v) for v in p) for p in params]
        elem = self.phi.element_size()
        self._arr = (L.AcInstance3D * len(self.shapes))()
        for i, ((nz, ny, nx), o, (h, dt, eps)) in enumerate(zip(self.shapes, self.offsets, self.params)):
            self._arr[i] = L.AcInstance3D(self.phi.data_ptr() + o * elem,
                                          self.work.data_ptr() + o * elem, nx, ny, nz, h, dt, eps)

    @property
    def cells(self) -> int:
        return sum(nx * ny * nz for (nz, ny, nx) in self.shapes)

    def views(self):
        return [self.phi[o:o + nz * ny * nx].view(nz, ny, nx)
                for o, (nz, ny, nx) in zip(self.offsets, self.shapes)]

    def step(self, nsteps: int, tune=None, stream=None) -> dict:
        info = L.AcBatchInfo()
        st = L.lib().ac_step_batched_3d(self._arr, len(self.shapes), int(nsteps),
                                        _dtype_code(self.phi), _tune(tune), ctypes.byref(info),
                                        _stream(stream))
        L.check(st, "ac_step_batched_3d")
        return info.as_dict()


def autotune2d(nx: int, ny: int, dtype=torch.float32, probe_steps: int = 200, stream=None) -> dict:
    best = L.AcTune()
    code = L.AC_F64 if dtype == torch.float64 else L.AC_F32
    L.check(L.lib().ac_autotune_2d(nx, ny, code, int(probe_steps), ctypes.byref(best),
                                   _stream(stream)), "ac_autotune_2d")
    return {k: getattr(best, k) for k, _ in best._fields_}


def autotune3d(nx: int, ny: int, nz: int, dtype=torch.float32, probe_steps: int = 50,
               stream=None) -> dict:
    best = L.AcTune()
    code = L.AC_F64 if dtype == torch.float64 else L.AC_F32
    L.check(L.lib().ac_autotune_3d(nx, ny, nz, code, int(probe_steps), ctypes.byref(best),
                                   _stream(stream)), "ac_autotune_3d")
    return {k: getattr(best, k) for k, _ in best._fields_}


def autotune(dim: int, dtype=torch.float32, cache_path: str | None = None) -> None:
    """ac_autotune: tune the representative grids of dimension dim, using and
    updating the JSON cache at cache_path when given."""
    code = L.AC_F64 if dtype == torch.float64 else L.AC_F32
    L.check(L.lib().ac_autotune(int(dim), code, cache_path.encode() if cache_path else None),
            "ac_autotune")


def tune_save(path: str) -> None:
    L.check(L.lib().ac_tune_save(path.encode()), "ac_tune_save")


def tune_load(path: str) -> None:
    L.check(L.lib().ac_tune_load(path.encode()), "ac_tune_load")


def tune_clear() -> None:
    L.lib().ac_tune_clear()


def judge2d(a: torch.Tensor, b: torch.Tensor, h: float, window: int = 3, stream=None):
    """(interface error, L2 error) per grid for [batch, ny, nx] FP32 device fields."""
    if a.shape != b.shape or a.dim() != 3 or a.dtype != torch.float32 or b.dtype != torch.float32:
        raise ValueError("two [batch, ny, nx] float32 tensors of one shape expected")
    if not (a.is_contiguous() and b.is_contiguous()):
        raise ValueError("contiguous tensors expected")
    n, ny, nx = a.shape
    iface = torch.empty(n, dtype=torch.float32, device=a.device)
    l2 = torch.empty(n, dtype=torch.float32, device=a.device)
    ws = torch.empty(int(L.lib().ac_judge_workspace_bytes(n)), dtype=torch.uint8, device=a.device)
    L.check(L.lib().ac_judge_2d(a.data_ptr(), b.data_ptr(), n, nx, ny, float(h), int(window),
                                iface.data_ptr(), l2.data_ptr(), ws.data_ptr(), _stream(stream)),
            "ac_judge_2d")
    return iface, l2


def err_trace(phi32: torch.Tensor, phi64: torch.Tensor, h: float, dt: float, eps: float,
              nsteps: int, stream=None):
    """Advance an FP32 and an FP64 copy of one grid together by nsteps steps,
    in place, and return (rms, err): rms[t] is the RMS difference of the two
    states after step t + 1 (a device FP64 tensor), err its mean -- the
    paper's Err (Eq. ERReq) between the two precisions."""
    if phi32.dtype != torch.float32 or phi64.dtype != torch.float64:
        raise TypeError("phi32 must be float32 and phi64 float64")
    if phi32.shape != phi64.shape or phi32.dim() not in (2, 3):
        raise ValueError("phi32 and phi64 must be 2D or 3D grids of one shape")
    _check_tensor(phi32, phi32.dim())
    _check_tensor(phi64, phi64.dim())
    w32, w64 = torch.empty_like(phi32), torch.empty_like(phi64)
    rms = torch.empty(max(int(nsteps), 1), dtype=torch.float64, device=phi32.device)
    err = torch.empty(1, dtype=torch.float64, device=phi32.device)
    if phi32.dim() == 2:
        ny, nx = phi32.shape
        st = L.lib().ac_err_2d(phi32.data_ptr(), w32.data_ptr(), phi64.data_ptr(), w64.data_ptr(),
                               nx, ny, float(h), float(dt), float(eps), int(nsteps),
                               rms.data_ptr(), err.data_ptr(), _stream(stream))
    else:
        nz, ny, nx = phi32.shape
        st = L.lib().ac_err_3d(phi32.data_ptr(), w32.data_ptr(), phi64.data_ptr(), w64.data_ptr(),
                               nx, ny, nz, float(h), float(dt), float(eps), int(nsteps),
                               rms.data_ptr(), err.data_ptr(), _stream(stream))
    L.check(st, "ac_err")
    return rms[:int(nsteps)], float(err.item())
