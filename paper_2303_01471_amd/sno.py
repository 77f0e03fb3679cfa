"""Python side of the spectral neural-operator surrogate (include/qhd_sno.h).

Argument marshalling only: the forward pass, the loss, the backward pass and
the Adam step all run in the HIP kernels of libqhd.so.  Device buffers and
streams come from PyTorch (ROCm build).
"""
from __future__ import annotations

import numpy as np

from . import qhd as q


class Surrogate:
    """One surrogate network on the current GPU.

    ``precision`` is "bf16" (BF16 weights/activations, FP32 accumulation) or
    "fp32" (FP32 throughout, for gradient checks).  ``train`` keeps the per-layer
    activations that ``backward`` needs."""

    def __init__(self, grid: int = 128, width: int = 32, modes: int = 16, layers: int = 4,
                 max_batch: int = 64, precision: str = "bf16", train: bool = True, seed: int = 0):
        prec = {"bf16": q.QHD_SNO_BF16, "fp32": q.QHD_SNO_FP32}[precision]
        self.desc = q.qhd_sno_desc(grid, width, modes, layers, max_batch, prec, 1 if train else 0, seed)
        self.grid, self.width, self.modes, self.layers = grid, width, modes, layers
        self.max_batch = max_batch
        self.handle = q.qhd_sno_create(self.desc)
        self.param_count = q.qhd_sno_param_count(self.handle)

    def get_params(self) -> np.ndarray:
        out = np.empty(self.param_count, dtype=np.float32)
        q.qhd_sno_get_params(self.handle, out.ctypes.data)
        return out

    def set_params(self, p: np.ndarray):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == self.param_count
        q.qhd_sno_set_params(self.handle, a.ctypes.data)

    def _check_f(self, f):
        import torch
        assert f.dtype == torch.float64 and f.is_cuda and f.is_contiguous()
        assert f.numel() % (self.grid * self.grid) == 0
        b = f.numel() // (self.grid * self.grid)
        assert 1 <= b <= self.max_batch
        return b

    def forward(self, f, out=None, stream=None):
        """f: FP64 CUDA tensor [B, S, S] -> density FP32 [B, S, S] (asynchronous)."""
        import torch
        b = self._check_f(f)
        if out is None:
            out = torch.empty((b, self.grid, self.grid), dtype=torch.float32, device=f.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == f.numel()
        q.qhd_sno_forward(self.handle, f.data_ptr(), b, out.data_ptr(), q._stream_handle(stream))
        return out

    def backward(self, f, rho_target, want_grad: bool = False, stream=None):
        """Forward + loss + backward.  Returns (loss, flat FP32 gradient or None)."""
        import torch
        b = self._check_f(f)
        assert rho_target.dtype == torch.float32 and rho_target.is_contiguous()
        assert rho_target.numel() == f.numel()
        g = np.empty(self.param_count, dtype=np.float32) if want_grad else None
        loss = q.qhd_sno_backward(self.handle, f.data_ptr(), rho_target.data_ptr(), b,
                                  g.ctypes.data if g is not None else 0, q._stream_handle(stream))
        return loss, g

    def step(self, lr: float, stream=None):
        q.qhd_sno_step(self.handle, float(lr), q._stream_handle(stream))

    def close(self):
        if getattr(self, "handle", None):
            q.qhd_sno_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
