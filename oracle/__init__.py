"""CPU oracle for the Allen-Cahn explicit stepper.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the GPU path.

* ``step2d`` / ``step3d`` / ``step_batched2d`` -- plain FP64 C loops
  (``ac_oracle.c``): the explicit scheme of section 2.1 (Eq. pytorchACeq) with
  the zero-Neumann boundary of section 2, 5-point in 2D, 7-point in 3D.
* ``brute`` -- the same scheme written as a dense matrix (graph Laplacian of
  the grid) in NumPy, for tiny grids.
* ``diagnostics`` -- energy, volume radius, interface crossings, Hausdorff
  distance, error norms and the paper's Err metric (Eq. ERReq).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_ac_oracle.so")
_SRC = os.path.join(_HERE, "ac_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "sur_oracle.c")]
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]

_lib = None


def build(force: bool = False) -> str:
    """Compile ac_oracle.c with gcc into oracle/_ac_oracle.so."""
    stale = not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(s) for s in _SRCS)
    if force or stale:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, *_SRCS, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        i64, dbl, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        pd = ctypes.POINTER(ctypes.c_double)
        lib.ora_step2d.argtypes = [pd, i64, i64, dbl, dbl, dbl, i64, i32]
        lib.ora_step2d.restype = i32
        lib.ora_step3d.argtypes = [pd, i64, i64, i64, dbl, dbl, dbl, i64, i32]
        lib.ora_step3d.restype = i32
        lib.ora_step_batched2d.argtypes = [ctypes.c_int32, ctypes.POINTER(pd),
                                           ctypes.POINTER(i64), ctypes.POINTER(i64),
                                           pd, pd, pd, i64, i32]
        lib.ora_step_batched2d.restype = i32
        lib.ora_cpus_available.argtypes = []
        lib.ora_cpus_available.restype = i32
        lib.sur_num_params.argtypes = [i32, i32, i32]
        lib.sur_num_params.restype = i64
        lib.sur_forward.argtypes = [pd, i32, i32, i32, pd, i32, i32, i32, pd]
        lib.sur_forward.restype = i32
        lib.sur_loss_grad.argtypes = [pd, i32, i32, i32, pd, pd, i32, i32, i32, pd, pd]
        lib.sur_loss_grad.restype = i32
        lib.sur_conv_fwd.argtypes = [pd, i32, i32, i32, i32, pd, pd, i32, i32, pd]
        lib.sur_conv_fwd.restype = None
        lib.sur_pool_fwd.argtypes = [pd, i32, i32, i32, i32, pd]
        lib.sur_pool_fwd.restype = None
        lib.sur_up_fwd.argtypes = [pd, i32, i32, i32, i32, pd]
        lib.sur_up_fwd.restype = None
        _lib = lib
    return _lib


def cpus_available() -> int:
    """CPUs this process may use (sched_getaffinity)."""
    return int(_load().ora_cpus_available())


def eps_m(h: float, m: float) -> float:
    """Eq. emvalue: the tanh profile tanh(x / (sqrt(2) eps_m)) rises from -0.9
    to +0.9 over m cells."""
    return h * m / (2.0 * math.sqrt(2.0) * math.atanh(0.9))


def _as_f64(phi) -> np.ndarray:
    return np.ascontiguousarray(np.array(phi, dtype=np.float64, copy=True))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def step2d(phi0, h: float, dt: float, eps: float, nsteps: int, threads: int = 1) -> np.ndarray:
    """nsteps explicit steps of a 2D field of shape (ny, nx); returns a new FP64 array."""
    a = _as_f64(phi0)
    if a.ndim != 2:
        raise ValueError("2D field expected, shape (ny, nx)")
    ny, nx = a.shape
    rc = _load().ora_step2d(_ptr(a), nx, ny, h, dt, eps, int(nsteps), int(threads))
    if rc != 0:
        raise ValueError("ora_step2d failed (%d)" % rc)
    return a


def step3d(phi0, h: float, dt: float, eps: float, nsteps: int, threads: int = 1) -> np.ndarray:
    """nsteps explicit steps of a 3D field of shape (nz, ny, nx)."""
    a = _as_f64(phi0)
    if a.ndim != 3:
        raise ValueError("3D field expected, shape (nz, ny, nx)")
    nz, ny, nx = a.shape
    rc = _load().ora_step3d(_ptr(a), nx, ny, nz, h, dt, eps, int(nsteps), int(threads))
    if rc != 0:
        raise ValueError("ora_step3d failed (%d)" % rc)
    return a


def step_batched2d(fields, hs, dts, epss, nsteps: int, threads: int = 1) -> list:
    """Independent 2D instances, each with its own (h, dt, eps)."""
    arrs = [_as_f64(f) for f in fields]
    n = len(arrs)
    pd = ctypes.POINTER(ctypes.c_double)
    ptrs = (pd * n)(*[_ptr(a) for a in arrs])
    nx = (ctypes.c_int64 * n)(*[a.shape[1] for a in arrs])
    ny = (ctypes.c_int64 * n)(*[a.shape[0] for a in arrs])
    hh = np.ascontiguousarray(hs, dtype=np.float64)
    dd = np.ascontiguousarray(dts, dtype=np.float64)
    ee = np.ascontiguousarray(epss, dtype=np.float64)
    rc = _load().ora_step_batched2d(n, ptrs, nx, ny, _ptr(hh), _ptr(dd), _ptr(ee),
                                    int(nsteps), int(threads))
    if rc != 0:
        raise ValueError("ora_step_batched2d failed (%d)" % rc)
    return arrs
