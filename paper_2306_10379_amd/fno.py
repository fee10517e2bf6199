"""ctypes binding of the warm-start network ABI (include/fno.h).

Argument marshalling only: the forward pass, loss, gradient and Adam step run in the HIP
kernels of libgsi.so (csrc/fno.hip); PyTorch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import gsi

EXPORTS = ["fno_param_count", "fno_create", "fno_set_params", "fno_get_params", "fno_forward", "fno_loss_grad",
           "fno_adam", "fno_last_error", "fno_destroy"]


class FnoConfig(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("modes", ctypes.c_int32), ("width", ctypes.c_int32),
                ("layers", ctypes.c_int32), ("p", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("bf16_weights", ctypes.c_int32)]


_ready = False


def load():
    global _ready
    L = gsi.load()
    if not _ready:
        vp, i32, P = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER
        L.fno_param_count.argtypes = [P(FnoConfig)]
        L.fno_param_count.restype = ctypes.c_int64
        L.fno_create.argtypes = [P(vp), P(FnoConfig), ctypes.c_uint64, vp]
        L.fno_create.restype = ctypes.c_int
        L.fno_set_params.argtypes = [vp, vp]
        L.fno_set_params.restype = ctypes.c_int
        L.fno_get_params.argtypes = [vp, vp]
        L.fno_get_params.restype = ctypes.c_int
        L.fno_forward.argtypes = [vp, vp, i32, vp, vp]
        L.fno_forward.restype = ctypes.c_int
        L.fno_loss_grad.argtypes = [vp, vp, vp, i32, P(ctypes.c_double), vp]
        L.fno_loss_grad.restype = ctypes.c_int
        L.fno_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
        L.fno_adam.restype = ctypes.c_int
        L.fno_last_error.argtypes = [vp]
        L.fno_last_error.restype = ctypes.c_char_p
        L.fno_destroy.argtypes = [vp]
        L.fno_destroy.restype = None
        _ready = True
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, shape):
    """The library takes raw float32 device pointers: check what it will read."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()) or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float32 device tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")


class Net:
    """Owns an fno handle. Tensors are float32 (float64 for forward(..., f64=True)) on the
    handle's device; V is (B, N*N), targets (B, N*N, p). bf16_weights: the passes read a
    bfloat16 copy of the float32 parameters (which Adam updates)."""

    def __init__(self, N=256, modes=24, width=20, layers=4, p=32, max_batch=16, seed=0, stream=None,
                 bf16_weights=False):
        import torch
        self.cfg = FnoConfig(N, modes, width, layers, p, max_batch, int(bool(bf16_weights)))
        self.L = load()
        self.count = int(self.L.fno_param_count(ctypes.byref(self.cfg)))
        if self.count < 0:
            raise gsi.GsiError(gsi.GSI_EINVAL, "invalid network configuration")
        self.h = ctypes.c_void_p()
        st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        s = self.L.fno_create(ctypes.byref(self.h), ctypes.byref(self.cfg), int(seed), ctypes.c_void_p(st))
        self._check(s)
        self.N, self.p, self.n = N, p, N * N

    def _check(self, s):
        if s != gsi.GSI_OK:
            msg = self.L.fno_last_error(self.h).decode() if self.h.value else "error"
            raise gsi.GsiError(s, msg)

    def get_params(self):
        import torch
        out = torch.empty(self.count, dtype=torch.float32, device="cuda")
        self._check(self.L.fno_get_params(self.h, _p(out)))
        return out

    def set_params(self, t):
        _need(t, "params", (self.count,))
        self._check(self.L.fno_set_params(self.h, _p(t)))

    def forward(self, V, f64=False):
        import torch
        B = V.shape[0]
        _need(V, "V", (B, self.n))
        out = torch.empty((B, self.n, self.p), dtype=torch.float64 if f64 else torch.float32, device=V.device)
        self._check(self.L.fno_forward(self.h, _p(V), B, None if f64 else _p(out), _p(out) if f64 else None))
        return out

    def loss_grad(self, V, Xs, want_grad=True):
        import torch
        B = V.shape[0]
        _need(V, "V", (B, self.n))
        _need(Xs, "Xs", (B, self.n, self.p))
        loss = (ctypes.c_double * B)()
        grad = torch.empty(self.count, dtype=torch.float32, device=V.device) if want_grad else None
        self._check(self.L.fno_loss_grad(self.h, _p(V), _p(Xs), B, loss, _p(grad)))
        return np.array(loss[:]), grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.L.fno_adam(self.h, lr, beta1, beta2, eps))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.fno_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
