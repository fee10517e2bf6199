"""ctypes binding of the libgsi C ABI (include/gsi.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of
libgsi.so. PyTorch provides device memory and the stream. Loading fails loudly when
the library has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsi.so")

GSI_OK, GSI_EINVAL, GSI_ENOMEM, GSI_EDEVICE, GSI_NOT_CONVERGED, GSI_BREAKDOWN, GSI_EUNSUPPORTED = range(7)
GSI_RSD, GSI_RCG, GSI_SI = 1, 2, 3
GSI_FP64, GSI_MIXED_FP32, GSI_MIXED_BF16 = 0, 1, 2

EXPORTS = [
    "gsi_options_default", "gsi_create", "gsi_create_stencil", "gsi_create_hermitian", "gsi_hermitian_results", "gsi_recompute_choice", "gsi_step", "gsi_solve", "gsi_residuals", "gsi_get_x",
    "gsi_set_x0", "gsi_set_values", "gsi_spmm", "gsi_spmm_lowp", "gsi_history", "gsi_counters", "gsi_pass_times", "gsi_destroy",
    "gsi_status_str", "gsi_last_error", "gsi_create_batched", "gsi_solve_batched", "gsi_batched_results",
    "gsi_batched_get_x", "gsi_batched_set_tuning", "gsi_batched_set_wait_limit", "gsi_batched_timeline", "gsi_batched_pass_times", "gsi_batched_last_error", "gsi_destroy_batched",
    "gsi_orthonormalize", "gsi_orthonormalize_noalloc", "gsi_batched_set_shapes", "gsi_stream_rates",
]
PASSES = ["grad", "dir", "spmm", "update", "reduce", "small", "linesearch", "refresh", "eig", "gram"]


class GsiCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


class GsiZcsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


class GsiStencil(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64), ("diag", ctypes.c_double),
                ("off", ctypes.c_double), ("diag_vec", ctypes.c_void_p)]


@dataclass
class Stencil:
    """Matrix-free 5/7-point operator: diagonal diag (+ diag_vec[r]), off at each grid
    neighbour; grid nx x ny x nz, x fastest."""
    nx: int
    ny: int = 1
    nz: int = 1
    diag: float = 0.0
    off: float = -1.0
    diag_vec: object = None  # host array or device tensor of n values, or None

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


class GsiOptions(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("which", ctypes.c_int32), ("method", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("recompute_ax", ctypes.c_int32), ("k_restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("switch_tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("explicit_c", ctypes.c_int32),
                ("stall_window", ctypes.c_int32), ("cheb_degree", ctypes.c_int32), ("cheb_lo", ctypes.c_double),
                ("cheb_hi", ctypes.c_double), ("cheb_top", ctypes.c_double), ("check_symmetric", ctypes.c_int32),
                ("x0_seed", ctypes.c_uint64)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgsi.so (raises if it is missing: build it with paper_2306_10379_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgsi.so not found at {path}; build it with `python -m paper_2306_10379_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname: loaded first, it is the one the
    # library binds to, so both use one runtime (loaded the other way round, the process would
    # hold two runtimes and the library's would find no device)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.gsi_options_default.argtypes = [P(GsiOptions)]
    L.gsi_options_default.restype = None
    L.gsi_create.argtypes = [P(vp), P(GsiCsr), P(GsiOptions), vp, vp]
    L.gsi_create.restype = ctypes.c_int
    L.gsi_create_stencil.argtypes = [P(vp), P(GsiStencil), P(GsiOptions), vp, vp]
    L.gsi_create_stencil.restype = ctypes.c_int
    L.gsi_create_hermitian.argtypes = [P(vp), P(GsiZcsr), P(GsiOptions), vp, vp]
    L.gsi_create_hermitian.restype = ctypes.c_int
    L.gsi_hermitian_results.argtypes = [vp, P(dbl), vp, P(dbl)]
    L.gsi_hermitian_results.restype = ctypes.c_int
    L.gsi_recompute_choice.argtypes = [vp, P(i32), P(dbl), P(dbl)]
    L.gsi_recompute_choice.restype = ctypes.c_int
    L.gsi_step.argtypes = [vp, i32]
    L.gsi_step.restype = ctypes.c_int
    L.gsi_solve.argtypes = [vp, P(i32)]
    L.gsi_solve.restype = ctypes.c_int
    L.gsi_residuals.argtypes = [vp, P(dbl), P(dbl), P(dbl), P(dbl)]
    L.gsi_residuals.restype = ctypes.c_int
    L.gsi_get_x.argtypes = [vp, vp]
    L.gsi_get_x.restype = ctypes.c_int
    L.gsi_set_x0.argtypes = [vp, vp]
    L.gsi_set_x0.restype = ctypes.c_int
    L.gsi_set_values.argtypes = [vp, vp]
    L.gsi_set_values.restype = ctypes.c_int
    L.gsi_spmm.argtypes = [vp, vp, vp]
    L.gsi_spmm.restype = ctypes.c_int
    L.gsi_spmm_lowp.argtypes = [vp, vp, vp]
    L.gsi_spmm_lowp.restype = ctypes.c_int
    L.gsi_history.argtypes = [vp, P(i32), P(dbl), P(dbl), P(dbl), P(dbl), P(dbl)]
    L.gsi_history.restype = ctypes.c_int
    L.gsi_counters.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(i32), P(i32), P(i32)]
    L.gsi_counters.restype = ctypes.c_int
    L.gsi_pass_times.argtypes = [vp, i32, P(dbl), P(i32)]
    L.gsi_pass_times.restype = ctypes.c_int
    L.gsi_destroy.argtypes = [vp]
    L.gsi_destroy.restype = None
    L.gsi_status_str.argtypes = [ctypes.c_int]
    L.gsi_status_str.restype = ctypes.c_char_p
    L.gsi_last_error.argtypes = [vp]
    L.gsi_last_error.restype = ctypes.c_char_p
    L.gsi_create_batched.argtypes = [P(vp), i32, P(GsiCsr), P(i32), P(GsiOptions), P(vp), vp]
    L.gsi_create_batched.restype = ctypes.c_int
    L.gsi_solve_batched.argtypes = [vp, P(i32), P(i32)]
    L.gsi_solve_batched.restype = ctypes.c_int
    L.gsi_batched_results.argtypes = [vp, i32, P(dbl), P(dbl), P(i32)]
    L.gsi_batched_results.restype = ctypes.c_int
    L.gsi_batched_get_x.argtypes = [vp, i32, vp]
    L.gsi_batched_get_x.restype = ctypes.c_int
    L.gsi_batched_set_tuning.argtypes = [vp, i32, i32, i32]
    L.gsi_batched_set_tuning.restype = ctypes.c_int
    L.gsi_batched_set_shapes.argtypes = [vp, P(i32)]
    L.gsi_batched_set_shapes.restype = ctypes.c_int
    L.gsi_batched_set_wait_limit.argtypes = [vp, dbl]
    L.gsi_batched_set_wait_limit.restype = ctypes.c_int
    L.gsi_batched_timeline.argtypes = [vp, P(dbl), P(dbl), P(dbl), P(i32), P(i32)]
    L.gsi_batched_timeline.restype = ctypes.c_int
    L.gsi_batched_pass_times.argtypes = [vp, P(dbl)]
    L.gsi_batched_pass_times.restype = ctypes.c_int
    L.gsi_batched_last_error.argtypes = [vp]
    L.gsi_batched_last_error.restype = ctypes.c_char_p
    L.gsi_destroy_batched.argtypes = [vp]
    L.gsi_destroy_batched.restype = None
    for name in ("gsi_orthonormalize", "gsi_orthonormalize_noalloc"):
        getattr(L, name).argtypes = [vp, i64, i32, vp]
        getattr(L, name).restype = ctypes.c_int
    L.gsi_stream_rates.argtypes = [vp, vp, i64, i32, P(dbl), vp]
    L.gsi_stream_rates.restype = ctypes.c_int
    _lib = L
    return L


class GsiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gsi status {status}: {msg}")
        self.status = status


def _dptr(t) -> int:
    return int(t.data_ptr())


def _need_shape(name, t, shape):
    """The C ABI takes raw device pointers: a tensor of the wrong size would be read or
    written out of bounds, so the binding checks every block against the sizes it stands for."""
    if tuple(t.shape) != tuple(shape) and not (t.dim() == 1 and t.numel() == int(np.prod(shape))):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def options(**kw) -> GsiOptions:
    o = GsiOptions()
    load().gsi_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def gsi_create(rowptr, colind, vals, n: int, X0, opt: GsiOptions, stream=None):
    """Create a handle. rowptr/colind int32, vals float64, X0 float64 n x p: device tensors."""
    import torch
    L = load()
    for name, t, dt in (("rowptr", rowptr, torch.int32), ("colind", colind, torch.int32),
                        ("vals", vals, torch.float64), ("X0", X0, torch.float64)):
        if t is None and name == "X0":
            continue  # drawn on the device from opt.x0_seed
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {dt} device tensor")
    _need_shape("rowptr", rowptr, (int(n) + 1,))
    _need_shape("vals", vals, (colind.numel(),))
    if X0 is not None and 1 <= opt.p <= 128 and int(n) >= 1:  # the library rejects other sizes first
        _need_shape("X0", X0, (int(n), int(opt.p)))
    csr = GsiCsr(n=int(n), nnz=int(colind.numel()), rowptr=_dptr(rowptr), colind=_dptr(colind), vals=_dptr(vals))
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    s = L.gsi_create(ctypes.byref(h), ctypes.byref(csr), ctypes.byref(opt),
                     ctypes.c_void_p(_dptr(X0) if X0 is not None else None), st)
    if s != GSI_OK:
        msg = L.gsi_last_error(h).decode() if h.value else L.gsi_status_str(s).decode()
        if h.value:
            L.gsi_destroy(h)
        raise GsiError(s, msg)
    return h


def gsi_create_stencil(S: Stencil, dvec, X0, opt: GsiOptions, stream=None):
    """Create a handle for a matrix-free stencil; dvec: float64 device tensor of n values or None."""
    import torch
    L = load()
    if X0 is not None and (not X0.is_cuda or X0.dtype != torch.float64 or not X0.is_contiguous()):
        raise TypeError("X0 must be a contiguous float64 device tensor")
    if dvec is not None and (not dvec.is_cuda or dvec.dtype != torch.float64 or dvec.numel() != S.n):
        raise TypeError("diag_vec must be a float64 device tensor of n values")
    if X0 is not None and 1 <= opt.p <= 128 and min(int(S.nx), int(S.ny), int(S.nz)) >= 1:
        _need_shape("X0", X0, (int(S.n), int(opt.p)))
    st_ = GsiStencil(nx=int(S.nx), ny=int(S.ny), nz=int(S.nz), diag=float(S.diag), off=float(S.off),
                     diag_vec=_dptr(dvec) if dvec is not None else None)
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    s = L.gsi_create_stencil(ctypes.byref(h), ctypes.byref(st_), ctypes.byref(opt),
                             ctypes.c_void_p(_dptr(X0) if X0 is not None else None), st)
    if s != GSI_OK:
        msg = L.gsi_last_error(h).decode() if h.value else L.gsi_status_str(s).decode()
        if h.value:
            L.gsi_destroy(h)
        raise GsiError(s, msg)
    return h


def _check(h, s, allowed=(GSI_OK,)):
    if s not in allowed:
        raise GsiError(s, load().gsi_last_error(h).decode())
    return s


def gsi_step(h, n_iter: int):
    return _check(h, load().gsi_step(h, int(n_iter)))


def gsi_solve(h):
    it = ctypes.c_int32(0)
    s = _check(h, load().gsi_solve(h, ctypes.byref(it)), (GSI_OK, GSI_NOT_CONVERGED))
    return s, it.value


def gsi_residuals(h, p: int):
    ritz = (ctypes.c_double * p)()
    res = (ctypes.c_double * p)()
    rho, phi = ctypes.c_double(), ctypes.c_double()
    _check(h, load().gsi_residuals(h, ritz, res, ctypes.byref(rho), ctypes.byref(phi)))
    return np.array(ritz[:]), np.array(res[:]), rho.value, phi.value


def gsi_get_x(h, out):
    return _check(h, load().gsi_get_x(h, ctypes.c_void_p(_dptr(out))))


def gsi_set_x0(h, X0):
    return _check(h, load().gsi_set_x0(h, ctypes.c_void_p(_dptr(X0))))


def gsi_set_values(h, vals):
    _check(h, load().gsi_set_values(h, _dptr(vals)))


def gsi_spmm(h, W, Z):
    return _check(h, load().gsi_spmm(h, ctypes.c_void_p(_dptr(W)), ctypes.c_void_p(_dptr(Z))))


def gsi_spmm_lowp(h, W, Z):
    return _check(h, load().gsi_spmm_lowp(h, ctypes.c_void_p(_dptr(W)), ctypes.c_void_p(_dptr(Z))))


def gsi_history(h, capacity: int):
    cnt = ctypes.c_int32(capacity)
    arrs = [(ctypes.c_double * max(capacity, 1))() for _ in range(5)]
    _check(h, load().gsi_history(h, ctypes.byref(cnt), *arrs))
    m = cnt.value
    keys = ["rho", "phi", "mu", "beta_pr", "ginf_rel"]
    return {k: np.array(a[:m]) for k, a in zip(keys, arrs)}


def gsi_counters(h):
    vals = [ctypes.c_int32() for _ in range(7)]
    _check(h, load().gsi_counters(h, *[ctypes.byref(v) for v in vals]))
    keys = ["iters", "spmm", "restarts", "refreshes", "null_steps", "low_iters", "eig_sweeps"]
    return {k: v.value for k, v in zip(keys, vals)}


def gsi_pass_times(h, enable: int = -1):
    ms = (ctypes.c_double * len(PASSES))()
    cnt = (ctypes.c_int32 * len(PASSES))()
    _check(h, load().gsi_pass_times(h, int(enable), ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PASSES)}


def gsi_destroy(h):
    if h is not None and h.value:
        load().gsi_destroy(h)


def stream_rates(nbytes: int = 1 << 31, reps: int = 10, stream=None) -> dict:
    """The device's copy, read and write rates (gsi_stream_rates) on two buffers of nbytes:
    {"copy": GB/s of read + write, "read": GB/s, "write": GB/s, "us": [copy, read, write]}."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    us = (ctypes.c_double * 3)()
    L = load()
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    s = L.gsi_stream_rates(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), int(a.numel() * 8),
                           int(reps), us, st)
    if s != GSI_OK:
        raise GsiError(s, L.gsi_status_str(s).decode())
    nb = a.numel() * 8
    del a, b
    return {"copy": 2 * nb / (us[0] * 1e-6) / 1e9, "read": nb / (us[1] * 1e-6) / 1e9,
            "write": nb / (us[2] * 1e-6) / 1e9, "us": [us[0], us[1], us[2]], "bytes": nb}


def orthonormalize(X, noalloc: bool = False, stream=None) -> int:
    """Two passes of Cholesky QR on the contiguous float64 device block X (n x p, in place)
    through gsi_orthonormalize, or gsi_orthonormalize_noalloc (static scratch, no device
    allocation). Returns the status (GSI_OK or GSI_BREAKDOWN); other statuses raise."""
    import torch
    if not X.is_cuda or X.dtype != torch.float64 or not X.is_contiguous() or X.dim() != 2:
        raise TypeError("X must be a contiguous float64 n x p device tensor")
    L = load()
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    fn = L.gsi_orthonormalize_noalloc if noalloc else L.gsi_orthonormalize
    s = fn(ctypes.c_void_p(_dptr(X)), int(X.shape[0]), int(X.shape[1]), st)
    if s not in (GSI_OK, GSI_BREAKDOWN):
        raise GsiError(s, L.gsi_status_str(s).decode())
    return s


@dataclass
class Result:
    status: int
    iters: int
    ritz: np.ndarray
    col_res: np.ndarray
    rho: float
    phi: float
    counters: dict


class Solver:
    """Convenience wrapper owning a handle. A is an inputs.CSR (host arrays, copied to the
    device) or a tuple (rowptr, colind, vals, n) of device tensors. X0 = None draws the start
    block on the device from the option x0_seed (gsi_create)."""

    def __init__(self, A, X0, p: int, device="cuda", **opts):
        import torch
        stencil = isinstance(A, Stencil)
        if stencil:
            n = A.n
            dvec = A.diag_vec
            if dvec is not None and not torch.is_tensor(dvec):
                dvec = torch.as_tensor(np.ascontiguousarray(dvec, dtype=np.float64), device=device)
        elif isinstance(A, tuple):
            rowptr, colind, vals, n = A
        else:
            rowptr = torch.as_tensor(np.asarray(A.rowptr, dtype=np.int32), device=device)
            colind = torch.as_tensor(np.asarray(A.colind, dtype=np.int32), device=device)
            vals = torch.as_tensor(np.asarray(A.vals, dtype=np.float64), device=device)
            n = A.n
        if X0 is not None and not torch.is_tensor(X0):
            X0 = torch.as_tensor(np.ascontiguousarray(X0, dtype=np.float64), device=device)
        self.n, self.p = int(n), int(p)
        method = opts.pop("method", "rcg")
        precision = opts.pop("precision", "fp64")
        opts["method"] = {"rsd": GSI_RSD, "rcg": GSI_RCG, "si": GSI_SI}[method] if isinstance(method, str) else method
        opts["precision"] = {"fp64": GSI_FP64, "mixed": GSI_MIXED_FP32, "fp32": GSI_MIXED_FP32,
                             "bf16": GSI_MIXED_BF16}[precision] \
            if isinstance(precision, str) else precision
        if opts.get("recompute_ax") == "auto":
            opts["recompute_ax"] = -1
        elif "recompute_ax" in opts and opts["recompute_ax"] != -1:
            opts["recompute_ax"] = int(bool(opts["recompute_ax"]))
        for b in ("use_graph", "explicit_c", "check_symmetric"):
            if b in opts:
                opts[b] = int(bool(opts[b]))
        self.opt = options(p=self.p, **opts)
        self.nnz = None if stencil else int(colind.numel())
        if stencil:
            self.h = gsi_create_stencil(A, dvec, X0, self.opt)
        else:
            self.h = gsi_create(rowptr, colind, vals, self.n, X0, self.opt)
        self.device = X0.device if X0 is not None else torch.device(device)

    def step(self, n_iter: int):
        gsi_step(self.h, n_iter)

    def solve(self) -> tuple[int, int]:
        return gsi_solve(self.h)

    def residuals(self):
        return gsi_residuals(self.h, self.p)

    def get_x(self):
        import torch
        out = torch.empty((self.n, self.p), dtype=torch.float64, device=self.device)
        gsi_get_x(self.h, out)
        return out

    def set_x0(self, X0):
        import torch
        if not torch.is_tensor(X0):
            X0 = torch.as_tensor(np.ascontiguousarray(X0, dtype=np.float64), device=self.device)
        X0 = X0.to(device=self.device, dtype=torch.float64).contiguous()
        _need_shape("X0", X0, (self.n, self.p))
        gsi_set_x0(self.h, X0)

    def set_values(self, vals):
        """New matrix values (same sparsity pattern; for a stencil, the n values of its
        diagonal term); the iteration restarts from the current basis (subspace tracking)."""
        import torch
        if not torch.is_tensor(vals):
            vals = torch.as_tensor(np.asarray(vals, dtype=np.float64), device=self.device)
        vals = vals.to(device=self.device, dtype=torch.float64).contiguous()
        # a CSR handle takes nnz values; a stencil handle the n values of its diagonal term
        _need_shape("vals", vals, (self.n if self.nnz is None else self.nnz,))
        gsi_set_values(self.h, vals)

    def spmm(self, W):
        import torch
        W = W.to(device=self.device, dtype=torch.float64).contiguous()
        _need_shape("W", W, (self.n, self.p))
        Z = torch.empty_like(W)
        gsi_spmm(self.h, W, Z)
        torch.cuda.synchronize()
        return Z

    def spmm_lowp(self, W):
        import torch
        W = W.to(device=self.device, dtype=torch.float64).contiguous()
        _need_shape("W", W, (self.n, self.p))
        Z = torch.empty_like(W)
        gsi_spmm_lowp(self.h, W, Z)
        torch.cuda.synchronize()
        return Z

    def recompute_choice(self):
        """(recompute_ax chosen, ms per iteration with the recursion, ms with RCG(+))."""
        r, a, b = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
        _check(self.h, load().gsi_recompute_choice(self.h, ctypes.byref(r), ctypes.byref(a), ctypes.byref(b)))
        return r.value, a.value, b.value

    def history(self, capacity: int | None = None):
        return gsi_history(self.h, capacity or (self.opt.max_iter + 2))

    def counters(self):
        return gsi_counters(self.h)

    def pass_times(self, enable: int = -1):
        return gsi_pass_times(self.h, enable)

    def run(self) -> Result:
        status, iters = self.solve()
        ritz, res, rho, phi = self.residuals()
        return Result(status, iters, ritz, res, rho, phi, self.counters())

    def close(self):
        gsi_destroy(self.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------------- batched


def _bcheck(h, s, allowed=(GSI_OK,)):
    if s not in allowed:
        raise GsiError(s, load().gsi_batched_last_error(h).decode())
    return s


def gsi_create_batched(mats, ps, X0s, opt: GsiOptions, stream=None):
    """mats: list of (rowptr int32, colind int32, vals float64, n) device tensors; ps: list of
    block sizes; X0s: list of n x p float64 device tensors."""
    import torch
    L = load()
    count = len(mats)
    if len(ps) != count or len(X0s) != count:
        raise ValueError("mats, ps and X0s must have the same length")
    csrs = (GsiCsr * count)()
    for i, (rp, ci, vv, n) in enumerate(mats):
        _need_shape(f"rowptr[{i}]", rp, (int(n) + 1,))
        _need_shape(f"vals[{i}]", vv, (ci.numel(),))
        if 1 <= int(ps[i]) <= 64 and int(n) >= 1:
            _need_shape(f"X0s[{i}]", X0s[i], (int(n), int(ps[i])))
        csrs[i] = GsiCsr(n=int(n), nnz=int(ci.numel()), rowptr=_dptr(rp), colind=_dptr(ci), vals=_dptr(vv))
    parr = (ctypes.c_int32 * count)(*[int(x) for x in ps])
    xarr = (ctypes.c_void_p * count)(*[_dptr(x) for x in X0s])
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    s = L.gsi_create_batched(ctypes.byref(h), count, csrs, parr, ctypes.byref(opt), xarr, st)
    if s != GSI_OK:
        msg = L.gsi_batched_last_error(h).decode() if h.value else L.gsi_status_str(s).decode()
        if h.value:
            L.gsi_destroy_batched(h)
        raise GsiError(s, msg)
    return h


def gsi_solve_batched(h, count: int):
    iters = (ctypes.c_int32 * count)()
    status = (ctypes.c_int32 * count)()
    s = _bcheck(h, load().gsi_solve_batched(h, iters, status), (GSI_OK, GSI_NOT_CONVERGED, GSI_BREAKDOWN))
    return s, np.array(iters[:]), np.array(status[:])


def gsi_batched_results(h, i: int, p: int):
    ritz = (ctypes.c_double * p)()
    rho = ctypes.c_double()
    rs = ctypes.c_int32()
    _bcheck(h, load().gsi_batched_results(h, int(i), ritz, ctypes.byref(rho), ctypes.byref(rs)))
    return np.array(ritz[:]), rho.value, rs.value


def gsi_batched_get_x(h, i: int, out):
    return _bcheck(h, load().gsi_batched_get_x(h, int(i), ctypes.c_void_p(_dptr(out))))


def gsi_batched_timeline(h, count: int):
    """Per-problem (begin_us, switch_us, end_us, iters_low, team) of the last solve."""
    b = (ctypes.c_double * count)()
    w = (ctypes.c_double * count)()
    e = (ctypes.c_double * count)()
    lo = (ctypes.c_int32 * count)()
    tm = (ctypes.c_int32 * count)()
    _bcheck(h, load().gsi_batched_timeline(h, b, w, e, lo, tm))
    return np.array(b[:]), np.array(w[:]), np.array(e[:]), np.array(lo[:]), np.array(tm[:])


def gsi_batched_pass_times(h, count: int):
    """count x len(PASSES) microseconds per pass of the last solve."""
    us = (ctypes.c_double * (count * len(PASSES)))()
    _bcheck(h, load().gsi_batched_pass_times(h, us))
    return np.array(us[:]).reshape(count, len(PASSES))


def gsi_destroy_batched(h):
    if h is not None and h.value:
        load().gsi_destroy_batched(h)


class BatchedSolver:
    """Owns a batched handle. mats: list of inputs.CSR (copied to the device); X0s: list of
    n x p arrays; ps: list of block sizes."""

    def __init__(self, mats, X0s, ps, device="cuda", **opts):
        import torch
        self._keep = []
        dev_mats = []
        for A in mats:
            rp = torch.as_tensor(np.asarray(A.rowptr, dtype=np.int32), device=device)
            ci = torch.as_tensor(np.asarray(A.colind, dtype=np.int32), device=device)
            vv = torch.as_tensor(np.asarray(A.vals, dtype=np.float64), device=device)
            dev_mats.append((rp, ci, vv, A.n))
        xs = [X.to(device=device, dtype=torch.float64).contiguous() if torch.is_tensor(X)
              else torch.as_tensor(np.ascontiguousarray(X, dtype=np.float64), device=device) for X in X0s]
        self._keep = [dev_mats, xs]
        self.ns = [A.n for A in mats]
        self.ps = [int(x) for x in ps]
        precision = opts.pop("precision", "fp32")
        opts["precision"] = {"fp64": GSI_FP64, "fp32": GSI_MIXED_FP32, "mixed": GSI_MIXED_FP32}[precision] \
            if isinstance(precision, str) else precision
        method = opts.pop("method", "rcg")
        opts["method"] = {"rsd": GSI_RSD, "rcg": GSI_RCG, "si": GSI_SI}[method] if isinstance(method, str) else method
        self.opt = options(**opts)
        self.device = device
        self.h = gsi_create_batched(dev_mats, self.ps, xs, self.opt)

    def solve(self):
        return gsi_solve_batched(self.h, len(self.ps))

    def results(self, i):
        return gsi_batched_results(self.h, i, self.ps[i])

    def timeline(self):
        return gsi_batched_timeline(self.h, len(self.ps))

    def set_tuning(self, tiles_per_member: int, recruit_step: int, check_every: int):
        _bcheck(self.h, load().gsi_batched_set_tuning(self.h, int(tiles_per_member), int(recruit_step),
                                                      int(check_every)))
        self.tuning_policy = (int(tiles_per_member), int(recruit_step), int(check_every))

    def set_wait_limit(self, seconds: float):
        _bcheck(self.h, load().gsi_batched_set_wait_limit(self.h, float(seconds)))

    def set_shapes(self, codes):
        """Per-problem tile-shape codes (gsi_batched_set_shapes; see tuning.shape_code)."""
        if len(codes) != len(self.ps):
            raise ValueError(f"need {len(self.ps)} shape codes, got {len(codes)}")
        arr = (ctypes.c_int32 * len(self.ps))(*[int(c) for c in codes])
        _bcheck(self.h, load().gsi_batched_set_shapes(self.h, arr))

    def pass_times(self):
        return gsi_batched_pass_times(self.h, len(self.ps))

    def get_x(self, i):
        import torch
        out = torch.empty((self.ns[i], self.ps[i]), dtype=torch.float64, device=self.device)
        gsi_batched_get_x(self.h, i, out)
        return out

    def close(self):
        gsi_destroy_batched(self.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                self.close()
        except Exception:
            pass


class HermitianSolver(Solver):
    """Complex Hermitian problem (gsi_create_hermitian). A: scipy sparse complex matrix (host;
    copied to the device), X0: n x p complex host array or complex128 device tensor. run()
    returns (status, iters, ritz (p,), X (n x p complex128 device tensor), rho)."""

    def __init__(self, A, X0, p: int, device="cuda", **opts):
        import torch
        import scipy.sparse as sps
        A = sps.csr_matrix(A)
        A.sort_indices()
        n = A.shape[0]
        self._rowptr = torch.as_tensor(A.indptr.astype(np.int32), device=device)
        self._colind = torch.as_tensor(A.indices.astype(np.int32), device=device)
        self._vals = torch.as_tensor(np.ascontiguousarray(A.data.astype(np.complex128)).view(np.float64),
                                     device=device)
        if torch.is_tensor(X0):
            X0r = torch.view_as_real(X0.to(device=device, dtype=torch.complex128).contiguous()).contiguous()
        else:
            X0r = torch.as_tensor(np.ascontiguousarray(np.asarray(X0, dtype=np.complex128)).view(np.float64),
                                  device=device)
        if A.shape[0] != A.shape[1]:
            raise ValueError(f"A must be square, got {A.shape}")
        _need_shape("X0 (real view)", X0r, (n, 2 * int(p)))
        method = opts.pop("method", "rcg")
        opts["method"] = {"rsd": GSI_RSD, "rcg": GSI_RCG}[method] if isinstance(method, str) else method
        for b in ("use_graph", "explicit_c", "check_symmetric"):
            if b in opts:
                opts[b] = int(bool(opts[b]))
        self.n, self.p = int(n), int(p)
        self.opt = options(p=self.p, **opts)
        L = load()
        z = GsiZcsr(n=self.n, nnz=int(A.nnz), rowptr=_dptr(self._rowptr), colind=_dptr(self._colind),
                    vals=_dptr(self._vals))
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        s = L.gsi_create_hermitian(ctypes.byref(h), ctypes.byref(z), ctypes.byref(self.opt),
                                   ctypes.c_void_p(_dptr(X0r)), st)
        if s != GSI_OK:
            msg = L.gsi_last_error(h).decode() if h.value else L.gsi_status_str(s).decode()
            if h.value:
                L.gsi_destroy(h)
            raise GsiError(s, msg)
        self.h = h
        self.device = self._rowptr.device

    # the handle holds the real embedding (2n x 2p): the real-block calls of the base class
    # would take blocks of the wrong size
    def set_x0(self, X0):
        raise GsiError(GSI_EUNSUPPORTED, "create a new HermitianSolver for a new start block")

    def set_values(self, vals):
        raise GsiError(GSI_EUNSUPPORTED, "create a new HermitianSolver for new values")

    def spmm(self, W):
        raise GsiError(GSI_EUNSUPPORTED, "spmm of the real embedding is not exposed")

    def spmm_lowp(self, W):
        raise GsiError(GSI_EUNSUPPORTED, "spmm of the real embedding is not exposed")

    def get_x(self):
        return self.results()[1]

    def residuals(self):
        raise GsiError(GSI_EUNSUPPORTED, "use results(): ritz values, complex basis and rho")

    def results(self):
        import torch
        ritz = (ctypes.c_double * self.p)()
        rho = ctypes.c_double()
        X = torch.empty((self.n, self.p, 2), dtype=torch.float64, device=self.device)
        _check(self.h, load().gsi_hermitian_results(self.h, ritz, ctypes.c_void_p(_dptr(X)), ctypes.byref(rho)))
        return np.array(ritz[:]), torch.view_as_complex(X), rho.value

    def run(self):
        status, iters = self.solve()
        ritz, X, rho = self.results()
        return status, iters, ritz, X, rho
