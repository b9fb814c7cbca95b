"""Python handle over the learned K-step surrogate of libac (ac_sur_*).

Marshalling only: every forward, loss, backward and Adam step runs in the
library's HIP kernels; torch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

K_STEPS = 100            # explicit steps the surrogate advances per call


def num_params() -> int:
    return int(L.lib().ac_sur_num_params())


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Surrogate:
    """Device state of one network: weights, Adam moments, activations for up
    to ``batch_max`` grids of ``hw`` x ``hw``."""

    def __init__(self, batch_max: int, hw: int, stream=None):
        self.batch_max, self.hw = int(batch_max), int(hw)
        h = ctypes.c_void_p()
        st = (stream or torch.cuda.current_stream()).cuda_stream
        L.check(L.lib().ac_sur_create(ctypes.byref(h), self.batch_max, self.hw, st), "ac_sur_create")
        self._h = h
        self.n = num_params()
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.t = 0

    def close(self):
        if self._h:
            L.lib().ac_sur_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream) -> None:
        L.check(L.lib().ac_sur_set_stream(self._h, stream.cuda_stream), "ac_sur_set_stream")

    def set_weights(self, w) -> None:
        a = np.ascontiguousarray(w, dtype=np.float32)
        L.check(L.lib().ac_sur_set_weights(self._h, _fptr(a), self.n), "ac_sur_set_weights")
        self.t = 0

    def get_weights(self) -> np.ndarray:
        a = np.empty(self.n, dtype=np.float32)
        L.check(L.lib().ac_sur_get_weights(self._h, _fptr(a), self.n), "ac_sur_get_weights")
        return a

    def grads(self) -> np.ndarray:
        a = np.empty(self.n, dtype=np.float32)
        L.check(L.lib().ac_sur_get_grads(self._h, _fptr(a), self.n), "ac_sur_get_grads")
        return a

    def _check(self, x: torch.Tensor) -> int:
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise TypeError("contiguous float32 device tensor expected")
        if x.dim() != 3 or x.shape[1] != self.hw or x.shape[2] != self.hw:
            raise ValueError("shape [batch, %d, %d] expected" % (self.hw, self.hw))
        return int(x.shape[0])

    def forward(self, phi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """out = phi + U(phi): the state K_STEPS explicit steps later, predicted."""
        b = self._check(phi)
        if out is None:
            out = torch.empty_like(phi)
        L.check(L.lib().ac_sur_forward(self._h, phi.data_ptr(), out.data_ptr(), b), "ac_sur_forward")
        return out

    def infer(self, phi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """forward() for inference: the head and residual run in the last
        layer's epilogue; no activations are kept for backward()."""
        b = self._check(phi)
        if out is None:
            out = torch.empty_like(phi)
        else:
            self._check(out)
            if out.data_ptr() == phi.data_ptr():
                raise ValueError("out must not alias phi")
        L.check(L.lib().ac_sur_infer(self._h, phi.data_ptr(), out.data_ptr(), b), "ac_sur_infer")
        return out

    def loss(self, target: torch.Tensor) -> torch.Tensor:
        b = self._check(target)
        L.check(L.lib().ac_sur_loss(self._h, target.data_ptr(), b, self._loss.data_ptr()), "ac_sur_loss")
        return self._loss

    def backward(self, batch: int, dloss_dout: torch.Tensor | None = None) -> None:
        """Parameter gradients after forward(): of the loss stored by loss(), or
        of any loss whose gradient with respect to the output is dloss_dout."""
        ptr = None
        if dloss_dout is not None:
            if self._check(dloss_dout) != int(batch):
                raise ValueError("dloss_dout must hold %d grids" % int(batch))
            ptr = dloss_dout.data_ptr()
        L.check(L.lib().ac_sur_backward(self._h, ptr, int(batch)), "ac_sur_backward")

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
        self.t += 1
        L.check(L.lib().ac_sur_adam_step(self._h, lr, b1, b2, eps, self.t), "ac_sur_adam_step")

    def train_step(self, phi: torch.Tensor, target: torch.Tensor, lr: float) -> torch.Tensor:
        self.forward(phi)
        loss = self.loss(target)
        self.backward(phi.shape[0])
        self.adam(lr)
        return loss
