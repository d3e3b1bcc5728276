"""Python binding of libnyspcg (randomized Nystrom PCG on MI355X / gfx950).

Argument marshalling only: every numerical step runs in the HIP kernels of
``csrc/`` behind the C ABI declared in ``include/nyspcg.h``.  PyTorch supplies
device memory and the current HIP stream.  The functions carry the C names.

If the shared library has not been built, every call raises ``RuntimeError``;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnyspcg.so")

NYS_OK, NYS_NOT_CONVERGED = 0, 1
NYS_ERR_ARG, NYS_ERR_NOT_PSD, NYS_ERR_BREAKDOWN, NYS_ERR_DEVICE, NYS_ERR_WORKSPACE = -1, -2, -3, -4, -5
NYS_F64, NYS_F32 = 0, 1
NYS_PREC_FP64, NYS_PREC_FP32, NYS_PREC_FP32_REFINE64, NYS_PREC_BF16X3_REFINE64 = 0, 1, 2, 3
NYS_OP_DENSE, NYS_OP_XTX, NYS_OP_RBF, NYS_OP_CALLBACK = 0, 1, 2, 3
NYS_ADA_ERR, NYS_ADA_ERR_LAM, NYS_ADA_RATIO = 0, 1, 2

EXPORTED = ["nys_workspace_size", "nys_gaussian", "nys_sketch", "nys_factor", "nys_op_apply",
            "nys_precond_apply", "nys_pcg_solve", "nys_pcg_solve_noalloc", "nys_noalloc_scratch_bytes",
            "nys_workspace_size_ragged", "nys_pcg_solve_ragged",
            "nys_pcg_backward", "nys_rbf_cross", "nys_workspace_size_adaptive", "nys_power_err_est",
            "nys_nystrom_adaptive", "nys_workspace_size_columns", "nys_sketch_columns",
            "nys_workspace_size_sketch_solve", "nys_sketch_solve", "nys_workspace_size_block",
            "nys_block_pcg_solve", "nys_workspace_size_weight_rows", "nys_weight_rows", "nys_timing_begin",
            "nys_timing_end", "nys_workspace_size_autotune", "nys_autotune", "nys_autotune_query",
            "nys_autotune_entries", "nys_autotune_clear", "nys_autotune_load", "nys_autotune_save",
            "nys_last_error", "nys_version"]


class NysError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("nyspcg status %d: %s" % (status, msg))
        self.status = status


# nys_apply_fn: int32 (*)(void* ctx, int64 k, int32 dtype, const void* V, int64 ldv, void* W, int64 ldw,
#                        void* stream)
APPLY_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p)


class _Operator(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_int64),
                ("data", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("sigma", ctypes.c_double), ("scale", ctypes.c_double),
                ("apply", APPLY_FN), ("ctx", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class _Precond(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ell", ctypes.c_int64), ("U", ctypes.c_void_p),
                ("ldu", ctypes.c_int64), ("dtype", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("lam", ctypes.c_void_p), ("nu", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("device_info", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(ctypes.c_int32)), ("relres", ctypes.POINTER(ctypes.c_double)),
                ("status", ctypes.POINTER(ctypes.c_int32)), ("refine_steps", ctypes.c_int32),
                ("total_iters", ctypes.c_int32)]


_lib = None


def lib():
    """Load libnyspcg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnyspcg.so is not built: run python -m paper_2110_02820_amd._build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        P = ctypes.POINTER
        L.nys_workspace_size.restype = sz
        L.nys_workspace_size.argtypes = [P(_Operator), i64, i64, i32]
        L.nys_gaussian.argtypes = [ctypes.c_uint64, i64, i64, vp, i64, vp]
        L.nys_sketch.argtypes = [P(_Operator), i64, ctypes.c_uint64, vp, vp, vp, i32, vp, sz, vp]
        L.nys_factor.argtypes = [vp, vp, P(_Precond), i32, vp, sz, vp]
        L.nys_op_apply.argtypes = [P(_Operator), dbl, vp, i64, i64, vp, i64, i32, vp, sz, vp]
        L.nys_precond_apply.argtypes = [P(_Precond), dbl, vp, i64, i64, vp, i64, vp, sz, vp]
        L.nys_pcg_solve.argtypes = [P(_Operator), P(_Precond), P(dbl), i64, vp, i64, i64, vp, i64,
                                    P(_Opts), P(_Info), vp, sz, vp]
        L.nys_pcg_solve_noalloc.argtypes = [P(_Operator), P(_Precond), P(dbl), i64, vp, i64, i64, vp, i64,
                                            P(_Opts), P(_Info), vp]
        L.nys_noalloc_scratch_bytes.restype = sz
        L.nys_noalloc_scratch_bytes.argtypes = []
        L.nys_workspace_size_autotune.restype = sz
        L.nys_workspace_size_autotune.argtypes = [P(_Operator), i64]
        L.nys_autotune.argtypes = [P(_Operator), i32, P(i64), i32, vp, sz, vp]
        L.nys_autotune_query.argtypes = [P(_Operator), i32, i64, P(i32), P(i32)]
        L.nys_autotune_entries.restype = i64
        L.nys_autotune_entries.argtypes = []
        L.nys_autotune_clear.argtypes = []
        L.nys_autotune_load.argtypes = [ctypes.c_char_p]
        L.nys_autotune_save.argtypes = [ctypes.c_char_p]
        L.nys_workspace_size_ragged.restype = sz
        L.nys_workspace_size_ragged.argtypes = [P(_Operator), P(_Precond), i32, i32]
        L.nys_pcg_solve_ragged.argtypes = [P(_Operator), P(_Precond), P(dbl), P(vp), P(vp), i32,
                                           P(_Opts), P(_Info), vp, sz, vp]
        L.nys_pcg_backward.argtypes = [P(_Operator), P(_Precond), dbl, vp, vp, vp, P(dbl), P(dbl), vp,
                                       P(_Opts), P(_Info), vp, sz, vp]
        L.nys_rbf_cross.argtypes = [P(_Operator), vp, i64, i64, i32, vp, vp, vp, P(dbl), vp, sz, vp]
        L.nys_workspace_size_adaptive.restype = sz
        L.nys_workspace_size_adaptive.argtypes = [P(_Operator), i64, i32]
        L.nys_power_err_est.argtypes = [P(_Operator), P(_Precond), i32, vp, P(dbl), i32, vp, sz, vp]
        L.nys_nystrom_adaptive.argtypes = [P(_Operator), i64, i64, i32, dbl, dbl, i32, ctypes.c_uint64, vp, vp,
                                           i64, P(_Precond), P(dbl), i32, vp, sz, vp]
        L.nys_workspace_size_columns.restype = sz
        L.nys_workspace_size_columns.argtypes = [P(_Operator), i64]
        L.nys_sketch_columns.argtypes = [P(_Operator), i64, vp, vp, vp, vp, sz, vp]
        L.nys_workspace_size_sketch_solve.restype = sz
        L.nys_workspace_size_sketch_solve.argtypes = [i64, i64, i64]
        L.nys_sketch_solve.argtypes = [P(_Precond), dbl, vp, i64, i64, vp, i64, vp, sz, vp]
        L.nys_timing_begin.argtypes = []
        L.nys_timing_end.argtypes = [P(dbl), P(i64)]
        L.nys_workspace_size_block.restype = sz
        L.nys_workspace_size_block.argtypes = [P(_Operator), i64, i64]
        L.nys_block_pcg_solve.argtypes = [P(_Operator), P(_Precond), dbl, vp, i64, i64, vp, i64, P(_Opts), P(_Info),
                                          vp, sz, vp]
        L.nys_workspace_size_weight_rows.restype = sz
        L.nys_workspace_size_weight_rows.argtypes = []
        L.nys_weight_rows.argtypes = [i64, i64, i32, vp, i64, vp, vp, i64, vp, sz, vp]
        for f in ("nys_gaussian", "nys_sketch", "nys_factor", "nys_op_apply", "nys_precond_apply",
                  "nys_pcg_solve", "nys_pcg_solve_noalloc", "nys_pcg_solve_ragged", "nys_pcg_backward", "nys_rbf_cross",
                  "nys_power_err_est", "nys_nystrom_adaptive", "nys_sketch_columns", "nys_sketch_solve",
                  "nys_block_pcg_solve", "nys_weight_rows", "nys_timing_begin", "nys_timing_end",
                  "nys_autotune", "nys_autotune_query", "nys_autotune_clear", "nys_autotune_load",
                  "nys_autotune_save"):
            getattr(L, f).restype = ctypes.c_int
        L.nys_last_error.restype = ctypes.c_char_p
        L.nys_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int, allow_not_converged: bool = False) -> int:
    if status == NYS_OK or (allow_not_converged and status == NYS_NOT_CONVERGED):
        return status
    raise NysError(status, lib().nys_last_error().decode())


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    return t.data_ptr()


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return NYS_F64
    if t.dtype == torch.float32:
        return NYS_F32
    raise ValueError("float32 or float64 data expected")


# --------------------------------------------------------------------------- operators

class _DeviceArray:
    """A device buffer described by the CUDA array interface, so that torch can
    view memory the library hands to a product routine without copying it."""

    def __init__(self, ptr: int, rows: int, cols: int, ld: int, dtype: torch.dtype):
        isz = 8 if dtype == torch.float64 else 4
        self.__cuda_array_interface__ = {
            "shape": (rows, cols), "typestr": "<f%d" % isz, "data": (int(ptr), False),
            "strides": (ld * isz, isz), "version": 2}


def device_view(ptr: int, rows: int, cols: int, ld: int, dtype: torch.dtype, device) -> torch.Tensor:
    """A rows x cols torch view (leading dimension ld) of device memory at ptr."""
    return torch.as_tensor(_DeviceArray(ptr, rows, cols, ld, dtype), device=device)


@dataclass
class Operator:
    """A (Section 1.1) as a dense matrix, ridge data X (A = scale X^T X), RBF
    points, or a caller's product routine (NYS_OP_CALLBACK)."""
    kind: int
    data: torch.Tensor
    n: int
    sigma: float = 0.0
    scale: float = 1.0
    fn: Optional[object] = None  # NYS_OP_CALLBACK: the ctypes product routine (kept alive here)
    weights: Optional[torch.Tensor] = None  # NYS_OP_XTX: float64 row weights d (A = scale X^T D X)

    @staticmethod
    def callback(apply, n: int, device="cuda", scale: float = 1.0) -> "Operator":
        """A given only through the product routine
        apply(k, dtype, V_ptr, ldv, W_ptr, ldw, stream_ptr) -> int, which enqueues
        W = A V (n x k blocks, NYS_F64 or NYS_F32 entries) on the given stream and
        returns 0 (the library adds scale and the shift)."""
        def raw(_ctx, k, dt, V, ldv, W, ldw, stream):
            try:
                return int(apply(int(k), int(dt), V, int(ldv), W, int(ldw), stream))
            except Exception:  # an exception must not cross the C frames
                return -1
        fn = APPLY_FN(raw)
        return Operator(NYS_OP_CALLBACK, torch.empty(1, dtype=torch.float64, device=device), int(n), scale=scale,
                        fn=fn)

    @staticmethod
    def from_function(f, n: int, device="cuda", scale: float = 1.0) -> "Operator":
        """A given as a torch function W = f(V) on n x k device tensors (float64,
        or float32 in the reduced-precision modes), run on the library call's
        stream."""
        dev = torch.device(device)

        def apply(k, dt, V, ldv, W, ldw, stream):
            dtype = torch.float64 if dt == NYS_F64 else torch.float32
            st = torch.cuda.ExternalStream(stream, device=dev) if stream else torch.cuda.default_stream(dev)
            with torch.cuda.stream(st):
                Vt = device_view(V, n, k, ldv, dtype, dev)
                Wt = device_view(W, n, k, ldw, dtype, dev)
                Wt.copy_(f(Vt))
            return 0
        return Operator.callback(apply, n, device, scale)

    @staticmethod
    def dense(A: torch.Tensor) -> "Operator":
        A = A.contiguous()
        return Operator(NYS_OP_DENSE, A, A.shape[0])

    @staticmethod
    def xtx(X: torch.Tensor, scale: float = 1.0) -> "Operator":
        X = X.contiguous()
        return Operator(NYS_OP_XTX, X, X.shape[1], scale=scale)

    @staticmethod
    def xtdx(X: torch.Tensor, d: torch.Tensor, scale: float = 1.0) -> "Operator":
        """A = scale X^T D X, D = diag(d), d >= 0 (finite): the X^T X operator with
        row weights, applied inside every product (float64 d in the float64
        products and residuals).  The weights are checked here."""
        d = d.reshape(-1).to(torch.float64).contiguous()
        if d.numel() != X.shape[0]:
            raise ValueError("xtdx: one weight per row of X")
        if not bool(torch.isfinite(d).all()) or bool((d < 0).any()):
            raise ValueError("xtdx: weights must be finite and >= 0")
        X = X.contiguous()
        return Operator(NYS_OP_XTX, X, X.shape[1], scale=scale, weights=d)

    @staticmethod
    def rbf(X: torch.Tensor, sigma: float, scale: float = 1.0) -> "Operator":
        X = X.contiguous()
        return Operator(NYS_OP_RBF, X, X.shape[0], sigma=float(sigma), scale=scale)

    def c(self) -> _Operator:
        d = self.data
        if self.kind == NYS_OP_CALLBACK:
            return _Operator(self.kind, NYS_F64, self.n, None, self.n, self.n, self.n, 0.0, self.scale, self.fn,
                             None, None)
        return _Operator(self.kind, _dt(d), self.n, _ptr(d), d.shape[0], d.shape[1], d.stride(0),
                         self.sigma, self.scale, APPLY_FN(), None, _ptr(self.weights))


@dataclass
class Precond:
    """Factored Nystrom approximation U diag(lam) U^T (mu-independent)."""
    U: torch.Tensor
    lam: torch.Tensor
    nu: float = 0.0

    def c(self) -> _Precond:
        return _Precond(self.U.shape[0], self.U.shape[1], _ptr(self.U), self.U.stride(0), _dt(self.U), 0,
                        _ptr(self.lam), self.nu)


def workspace(op: Operator, ell: int, ncols: int = 1, prec: int = NYS_PREC_FP64) -> torch.Tensor:
    nb = lib().nys_workspace_size(ctypes.byref(op.c()), ell, ncols, prec)
    if nb == 0:
        raise NysError(NYS_ERR_ARG, "invalid operator for workspace sizing")
    return torch.empty(nb, dtype=torch.uint8, device=op.data.device)


def _ws(op, ell, ncols, prec, ws):
    return ws if ws is not None else workspace(op, ell, ncols, prec)


def _ws_shape(n: int, ell: int, ncols: int, device) -> torch.Tensor:
    """Workspace for calls that only depend on (n, ell): size it with a dense
    descriptor whose data pointer is a non-null placeholder (never read)."""
    fake = _Operator(NYS_OP_DENSE, NYS_F64, n, 1, n, n, n, 0.0, 1.0)
    nb = lib().nys_workspace_size(ctypes.byref(fake), ell, ncols, NYS_PREC_FP64)
    return torch.empty(nb, dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------- entry points

def nys_gaussian(seed: int, n: int, ell: int, device="cuda") -> torch.Tensor:
    out = torch.empty(n, ell, dtype=torch.float64, device=device)
    _check(lib().nys_gaussian(seed, n, ell, _ptr(out), ell, _stream()))
    return out


def nys_sketch(op: Operator, ell: int, seed: int = 0, omega0: Optional[torch.Tensor] = None,
               prec: int = NYS_PREC_FP64, ws: Optional[torch.Tensor] = None):
    dev = op.data.device
    Om = torch.empty(op.n, ell, dtype=torch.float64, device=dev)
    Y = torch.empty(op.n, ell, dtype=torch.float64, device=dev)
    if omega0 is not None:
        omega0 = omega0.to(device=dev, dtype=torch.float64).contiguous()
    w = _ws(op, ell, 1, prec, ws)
    _check(lib().nys_sketch(ctypes.byref(op.c()), ell, seed, _ptr(omega0), _ptr(Om), _ptr(Y), prec,
                            _ptr(w), w.numel(), _stream()))
    return Om, Y


def nys_factor(Omega: torch.Tensor, Y: torch.Tensor, dtype=torch.float64,
               ws: Optional[torch.Tensor] = None, op: Optional[Operator] = None,
               prec: int = NYS_PREC_FP64) -> Precond:
    """Shifted Cholesky + SVD factorisation of a sketch; prec is the arithmetic
    the sketch was computed in (it sets the minimum shift)."""
    n, ell = Y.shape
    U = torch.empty(n, ell, dtype=dtype, device=Y.device)
    lam = torch.empty(ell, dtype=torch.float64, device=Y.device)
    p = _Precond(n, ell, _ptr(U), ell, NYS_F64 if dtype == torch.float64 else NYS_F32, 0, _ptr(lam), 0.0)
    if ws is None:
        ws = _ws_shape(n, ell, 1, Y.device) if op is None else workspace(op, ell)
    _check(lib().nys_factor(_ptr(Omega), _ptr(Y), ctypes.byref(p), prec, _ptr(ws), ws.numel(), _stream()))
    return Precond(U, lam, p.nu)


def nys_weight_rows(X: torch.Tensor, d: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """D^{1/2} X for weights d >= 0, one per row of X (float64 or float32 X);
    out may be X itself (in place)."""
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a row-major 2-D tensor")
    d = d.to(device=X.device, dtype=torch.float64).contiguous()
    if d.numel() != X.shape[0]:
        raise ValueError("need one weight per row of X")
    if out is None:
        out = torch.empty_like(X, memory_format=torch.contiguous_format)
    elif out.shape != X.shape or out.dtype != X.dtype or out.device != X.device or out.stride(1) != 1:
        raise ValueError("out must be a row-major tensor of X's shape, dtype and device")
    ws = torch.empty(lib().nys_workspace_size_weight_rows(), dtype=torch.uint8, device=X.device)
    _check(lib().nys_weight_rows(X.shape[0], X.shape[1], _dt(X), _ptr(X), X.stride(0), _ptr(d), _ptr(out),
                                 out.stride(0), _ptr(ws), ws.numel(), _stream()))
    return out


def nys_sketch_solve(P: Precond, mu: float, B: torch.Tensor, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Nystrom sketch-and-solve: (U diag(lam) U^T + mu I)^{-1} B (Woodbury);
    an approximation of (A + mu I)^{-1} B only as good as A_hat is."""
    B2 = B.reshape(B.shape[0], -1).to(torch.float64).contiguous()
    n, k = B2.shape
    X = torch.empty_like(B2)
    if ws is None:
        ws = torch.empty(lib().nys_workspace_size_sketch_solve(n, P.U.shape[1], k), dtype=torch.uint8,
                         device=B2.device)
    _check(lib().nys_sketch_solve(ctypes.byref(P.c()), float(mu), _ptr(B2), k, k, _ptr(X), k, _ptr(ws), ws.numel(),
                                  _stream()))
    return X.reshape(B.shape)


def nys_sketch_columns(op: Operator, idx, ws: Optional[torch.Tensor] = None):
    """Column-sampling sketch: Omega = I[:, idx], Y = A[:, idx] (float64).
    idx: ell distinct indices (any int sequence or tensor)."""
    dev = op.data.device
    idx_t = torch.as_tensor(idx, dtype=torch.int64).to(dev).contiguous()
    ell = idx_t.numel()
    Om = torch.empty(op.n, ell, dtype=torch.float64, device=dev)
    Y = torch.empty(op.n, ell, dtype=torch.float64, device=dev)
    if ws is None:
        nb = lib().nys_workspace_size_columns(ctypes.byref(op.c()), ell)
        if nb == 0:
            raise NysError(NYS_ERR_ARG, "invalid operator for workspace sizing")
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(lib().nys_sketch_columns(ctypes.byref(op.c()), ell, _ptr(idx_t), _ptr(Om), _ptr(Y), _ptr(ws),
                                    ws.numel(), _stream()))
    return Om, Y


def workspace_adaptive(op: Operator, ell_max: int, prec: int = NYS_PREC_FP64) -> torch.Tensor:
    nb = lib().nys_workspace_size_adaptive(ctypes.byref(op.c()), ell_max, prec)
    if nb == 0:
        raise NysError(NYS_ERR_ARG, "invalid operator for workspace sizing")
    return torch.empty(nb, dtype=torch.uint8, device=op.data.device)


def nys_power_err_est(op: Operator, P: Precond, q: int, g: Optional[torch.Tensor] = None, seed: int = 0,
                      prec: int = NYS_PREC_FP64, ws: Optional[torch.Tensor] = None) -> float:
    """Randomized power estimate of ||A - U diag(lam) U^T|| after q steps from
    the start vector g (drawn with nys_gaussian(seed, n, 1) when None)."""
    if g is None:
        g = nys_gaussian(seed, op.n, 1, device=op.data.device)
    g = g.to(device=op.data.device, dtype=torch.float64).contiguous()
    w = ws if ws is not None else workspace_adaptive(op, P.U.shape[1], prec)
    est = ctypes.c_double(0.0)
    _check(lib().nys_power_err_est(ctypes.byref(op.c()), ctypes.byref(P.c()), q, _ptr(g), ctypes.byref(est), prec,
                                   _ptr(w), w.numel(), _stream()))
    return est.value


def nys_nystrom_adaptive(op: Operator, ell0: int, ell_max: int, mu: float, tau: float = 44.0, q: int = 10,
                         criterion: int = NYS_ADA_ERR, seed: int = 0, prec: int = NYS_PREC_FP64,
                         dtype=torch.float64, ws: Optional[torch.Tensor] = None):
    """Adaptive rank selection: doubles the sketch size from ell0 until the
    criterion holds with tol = tau * mu (or ell_max is reached).  Returns
    (Precond, info) with info = {"ell", "err", "capped", "Omega", "Y"}."""
    dev = op.data.device
    n = op.n
    Om = torch.empty(n, ell_max, dtype=torch.float64, device=dev)
    Y = torch.empty(n, ell_max, dtype=torch.float64, device=dev)
    U = torch.empty(n, ell_max, dtype=dtype, device=dev)
    lam = torch.empty(ell_max, dtype=torch.float64, device=dev)
    p = _Precond(n, ell_max, _ptr(U), ell_max, NYS_F64 if dtype == torch.float64 else NYS_F32, 0, _ptr(lam), 0.0)
    w = ws if ws is not None else workspace_adaptive(op, ell_max, prec)
    err = ctypes.c_double(0.0)
    st = _check(lib().nys_nystrom_adaptive(ctypes.byref(op.c()), ell0, ell_max, q, float(tau), float(mu), criterion,
                                           seed, _ptr(Om), _ptr(Y), ell_max, ctypes.byref(p), ctypes.byref(err),
                                           prec, _ptr(w), w.numel(), _stream()), allow_not_converged=True)
    ell = int(p.ell)
    P = Precond(U[:, :ell].contiguous(), lam[:ell].clone(), p.nu)
    return P, {"ell": ell, "err": err.value, "capped": st == NYS_NOT_CONVERGED,
               "Omega": Om[:, :ell], "Y": Y[:, :ell]}


def nys_op_apply(op: Operator, mu: float, V: torch.Tensor, ws: Optional[torch.Tensor] = None,
                 prec: Optional[int] = None) -> torch.Tensor:
    """(A + mu I) V.  float64 V computes in float64; float32 V in float32 (RBF:
    Gram tiles in float32, or bf16x3 with prec=NYS_PREC_BF16X3_REFINE64)."""
    V2 = V.reshape(V.shape[0], -1).contiguous()
    k = V2.shape[1]
    Z = torch.empty_like(V2)
    if prec is None:
        prec = NYS_PREC_FP64 if V2.dtype == torch.float64 else NYS_PREC_FP32
    w = _ws(op, 1, k, prec, ws)
    _check(lib().nys_op_apply(ctypes.byref(op.c()), float(mu), _ptr(V2), k, k, _ptr(Z), k, prec, _ptr(w),
                              w.numel(), _stream()))
    return Z.reshape(V.shape)


def nys_precond_apply(P: Precond, mu: float, R: torch.Tensor, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    R2 = R.reshape(R.shape[0], -1).contiguous().to(torch.float64)
    k = R2.shape[1]
    Z = torch.empty_like(R2)
    if ws is None:
        ws = _ws_shape(P.U.shape[0], P.U.shape[1], k, R.device)
    _check(lib().nys_precond_apply(ctypes.byref(P.c()), float(mu), _ptr(R2), k, k, _ptr(Z), k, _ptr(ws),
                                   ws.numel(), _stream()))
    return Z.reshape(R.shape)


@dataclass
class SolveInfo:
    iters: list
    relres: list
    status: list
    refine_steps: int
    total_iters: int
    code: int


def _opts(tol, maxit, prec, max_refine, check_every, inner_tol, device_info=0):
    return _Opts(tol, maxit, prec, max_refine, check_every, inner_tol, device_info, 0)


def nys_pcg_solve(op: Operator, P: Precond, mu, B: torch.Tensor, X0: Optional[torch.Tensor] = None,
                  tol: float = 1e-10, maxit: int = 500, prec: int = NYS_PREC_FP64, max_refine: int = 10,
                  check_every: int = 0, inner_tol: float = 1e-4, ws: Optional[torch.Tensor] = None,
                  raise_on_not_converged: bool = False):
    """Solve (A + mu_m I) X[:, m*nrhs + r] = B[:, r] for every mu_m.  Returns (X, SolveInfo)."""
    mus = [float(m) for m in (mu if isinstance(mu, (list, tuple)) else [mu])]
    B2 = B.reshape(B.shape[0], -1).contiguous().to(torch.float64)
    nrhs = B2.shape[1]
    k = len(mus) * nrhs
    if X0 is None:
        X = torch.zeros(B2.shape[0], k, dtype=torch.float64, device=B.device)
    else:
        X = X0.reshape(B2.shape[0], k).to(torch.float64).contiguous().clone()
    w = _ws(op, P.U.shape[1], k, prec, ws)
    it = (ctypes.c_int32 * k)()
    rr = (ctypes.c_double * k)()
    st = (ctypes.c_int32 * k)()
    info = _Info(it, rr, st, 0, 0)
    mu_arr = (ctypes.c_double * len(mus))(*mus)
    o = _opts(tol, maxit, prec, max_refine, check_every, inner_tol)
    code = lib().nys_pcg_solve(ctypes.byref(op.c()), ctypes.byref(P.c()), mu_arr, len(mus), _ptr(B2), nrhs,
                               nrhs, _ptr(X), k, ctypes.byref(o), ctypes.byref(info), _ptr(w), w.numel(),
                               _stream())
    _check(code, allow_not_converged=not raise_on_not_converged)
    si = SolveInfo(list(it), list(rr), list(st), info.refine_steps, info.total_iters, code)
    if B.dim() == 1 and k == 1:
        X = X.reshape(-1)
    return X, si


def nys_pcg_solve_device(op: Operator, P: Precond, mu, B: torch.Tensor, X: torch.Tensor, iters: torch.Tensor,
                         relres: torch.Tensor, status: torch.Tensor, tol: float = 1e-10, maxit: int = 500,
                         prec: int = NYS_PREC_FP64, max_refine: int = 10, inner_tol: float = 1e-4,
                         ws: Optional[torch.Tensor] = None):
    """Device-info form of nys_pcg_solve (opts.device_info = 1): nothing is read
    back and the stream is never synchronised, so the call can be captured into
    a graph.  B: n x nrhs float64, X: n x (nmu*nrhs) float64 (in: x0, out: x),
    both contiguous; iters (int32), relres (float64), status (int32): device
    tensors of nmu*nrhs entries written by the call's last kernels.  Runs exactly
    maxit iterations (refinement modes: max_refine steps of maxit).  Returns
    (refine_steps, total_iters), the fixed counts."""
    mus = [float(m) for m in (mu if isinstance(mu, (list, tuple)) else [mu])]
    if B.dtype != torch.float64 or X.dtype != torch.float64 or not B.is_contiguous() or not X.is_contiguous():
        raise ValueError("B and X must be contiguous float64 device tensors")
    B2 = B.reshape(B.shape[0], -1)
    nrhs = B2.shape[1]
    k = len(mus) * nrhs
    if X.numel() != B2.shape[0] * k:
        raise ValueError("X must have n x (nmu * nrhs) entries")
    for t, dt in ((iters, torch.int32), (relres, torch.float64), (status, torch.int32)):
        if t.dtype != dt or t.numel() < k or not t.is_cuda:
            raise ValueError("iters / relres / status: device tensors of int32 / float64 / int32, %d entries" % k)
    w = _ws(op, P.U.shape[1], k, prec, ws)
    info = _Info(ctypes.cast(ctypes.c_void_p(iters.data_ptr()), ctypes.POINTER(ctypes.c_int32)),
                 ctypes.cast(ctypes.c_void_p(relres.data_ptr()), ctypes.POINTER(ctypes.c_double)),
                 ctypes.cast(ctypes.c_void_p(status.data_ptr()), ctypes.POINTER(ctypes.c_int32)), 0, 0)
    mu_arr = (ctypes.c_double * len(mus))(*mus)
    o = _opts(tol, maxit, prec, max_refine, 1, inner_tol, device_info=1)
    _check(lib().nys_pcg_solve(ctypes.byref(op.c()), ctypes.byref(P.c()), mu_arr, len(mus), _ptr(B2), nrhs, nrhs,
                               _ptr(X), k, ctypes.byref(o), ctypes.byref(info), _ptr(w), w.numel(), _stream()))
    return info.refine_steps, info.total_iters


def nys_pcg_solve_noalloc(op: Operator, P: Precond, mu, B: torch.Tensor, X: torch.Tensor, iters: torch.Tensor,
                          relres: torch.Tensor, status: torch.Tensor, tol: float = 1e-10, maxit: int = 500,
                          prec: int = NYS_PREC_FP64, max_refine: int = 10, inner_tol: float = 1e-4):
    """Allocation-free form of nys_pcg_solve_device: the same call without a
    workspace (the library's static per-GPU scratch serves instead; calls that
    overlap on one GPU race).  Returns (refine_steps, total_iters)."""
    mus = [float(m) for m in (mu if isinstance(mu, (list, tuple)) else [mu])]
    if B.dtype != torch.float64 or X.dtype != torch.float64 or not B.is_contiguous() or not X.is_contiguous():
        raise ValueError("B and X must be contiguous float64 device tensors")
    B2 = B.reshape(B.shape[0], -1)
    nrhs = B2.shape[1]
    k = len(mus) * nrhs
    if X.numel() != B2.shape[0] * k:
        raise ValueError("X must have n x (nmu * nrhs) entries")
    for t, dt in ((iters, torch.int32), (relres, torch.float64), (status, torch.int32)):
        if t.dtype != dt or t.numel() < k or not t.is_cuda:
            raise ValueError("iters / relres / status: device tensors of int32 / float64 / int32, %d entries" % k)
    info = _Info(ctypes.cast(ctypes.c_void_p(iters.data_ptr()), ctypes.POINTER(ctypes.c_int32)),
                 ctypes.cast(ctypes.c_void_p(relres.data_ptr()), ctypes.POINTER(ctypes.c_double)),
                 ctypes.cast(ctypes.c_void_p(status.data_ptr()), ctypes.POINTER(ctypes.c_int32)), 0, 0)
    mu_arr = (ctypes.c_double * len(mus))(*mus)
    o = _opts(tol, maxit, prec, max_refine, 1, inner_tol, device_info=1)
    _check(lib().nys_pcg_solve_noalloc(ctypes.byref(op.c()), ctypes.byref(P.c()), mu_arr, len(mus), _ptr(B2), nrhs,
                                       nrhs, _ptr(X), k, ctypes.byref(o), ctypes.byref(info), _stream()))
    return info.refine_steps, info.total_iters


def nys_autotune(op: Operator, prec: int, ks: Sequence[int], ws: Optional[torch.Tensor] = None) -> None:
    """Time every tile shape of the reduced-precision RBF block product for each
    column count in ks on this operator and record the fastest (process-wide
    table; saved to $NYS_AUTOTUNE_CACHE when set)."""
    ks = [int(k) for k in ks]
    if ws is None:
        nb = lib().nys_workspace_size_autotune(ctypes.byref(op.c()), max(ks))
        if nb == 0:
            _check(NYS_ERR_ARG)
        ws = torch.empty(nb, dtype=torch.uint8, device=op.data.device)
    arr = (ctypes.c_int64 * len(ks))(*ks)
    _check(lib().nys_autotune(ctypes.byref(op.c()), prec, arr, len(ks), _ptr(ws), ws.numel(), _stream()))


def nys_autotune_query(op: Operator, prec: int, k: int):
    """(register kernel?, 16-column tiles per workgroup, workgroups per CU, 16-row
    fragments per wave, tuned?) of a k-column product."""
    ch = (ctypes.c_int32 * 4)()
    tuned = ctypes.c_int32(0)
    _check(lib().nys_autotune_query(ctypes.byref(op.c()), prec, k, ch, ctypes.byref(tuned)))
    return bool(ch[0]), int(ch[1]), int(ch[2]), int(ch[3]), bool(tuned.value)


def nys_autotune_entries() -> int:
    return int(lib().nys_autotune_entries())


def nys_autotune_clear() -> None:
    _check(lib().nys_autotune_clear())


def nys_autotune_load(path: str) -> None:
    _check(lib().nys_autotune_load(str(path).encode()))


def nys_autotune_save(path: str) -> None:
    _check(lib().nys_autotune_save(str(path).encode()))


def timing_begin() -> None:
    """Start timing launches of the X^T X product kernel with HIP events."""
    _check(lib().nys_timing_begin())


def timing_end():
    """Stop timing; returns (mean launch duration in ms, launches timed)."""
    avg = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().nys_timing_end(ctypes.byref(avg), ctypes.byref(cnt)))
    return avg.value, cnt.value


def nys_block_pcg_solve(op: Operator, P: Precond, mu: float, B: torch.Tensor, tol: float = 1e-10, maxit: int = 500,
                        check_every: int = 0, ws: Optional[torch.Tensor] = None, raise_on_not_converged: bool = False):
    """Coupled block PCG (O'Leary) for (A + mu I) X = B, float64, s <= 64
    columns sharing one block Krylov space.  Returns (X, SolveInfo)."""
    B2 = B.reshape(B.shape[0], -1).contiguous().to(torch.float64)
    n, s = B2.shape
    X = torch.empty_like(B2)
    if ws is None:
        nb = lib().nys_workspace_size_block(ctypes.byref(op.c()), P.U.shape[1], s)
        if nb == 0:
            raise NysError(NYS_ERR_ARG, "block PCG: 1 <= s <= 64 columns and a valid operator are required")
        ws = torch.empty(nb, dtype=torch.uint8, device=B2.device)
    it = (ctypes.c_int32 * s)()
    rr = (ctypes.c_double * s)()
    st = (ctypes.c_int32 * s)()
    info = _Info(it, rr, st, 0, 0)
    o = _opts(tol, maxit, NYS_PREC_FP64, 0, check_every, 0.0)
    code = lib().nys_block_pcg_solve(ctypes.byref(op.c()), ctypes.byref(P.c()), float(mu), _ptr(B2), s, s, _ptr(X), s,
                                     ctypes.byref(o), ctypes.byref(info), _ptr(ws), ws.numel(), _stream())
    _check(code, allow_not_converged=not raise_on_not_converged)
    return X.reshape(B.shape), SolveInfo(list(it), list(rr), list(st), info.refine_steps, info.total_iters, code)


def nys_pcg_solve_ragged(ops: Sequence[Operator], Ps: Sequence[Precond], mus: Sequence[float],
                         Bs: Sequence[torch.Tensor], tol: float = 1e-10, maxit: int = 500,
                         prec: int = NYS_PREC_FP64, max_refine: int = 10, check_every: int = 0,
                         inner_tol: float = 1e-4, ws: Optional[torch.Tensor] = None):
    npb = len(ops)
    cops = (_Operator * npb)(*[o.c() for o in ops])
    cps = (_Precond * npb)(*[p.c() for p in Ps])
    mu_arr = (ctypes.c_double * npb)(*[float(m) for m in mus])
    Bs = [b.reshape(-1).contiguous().to(torch.float64) for b in Bs]
    Xs = [torch.zeros_like(b) for b in Bs]
    barr = (ctypes.c_void_p * npb)(*[_ptr(b) for b in Bs])
    xarr = (ctypes.c_void_p * npb)(*[_ptr(x) for x in Xs])
    if ws is None:
        nb = lib().nys_workspace_size_ragged(cops, cps, npb, prec)
        ws = torch.empty(nb, dtype=torch.uint8, device=Bs[0].device)
    it = (ctypes.c_int32 * npb)()
    rr = (ctypes.c_double * npb)()
    st = (ctypes.c_int32 * npb)()
    info = _Info(it, rr, st, 0, 0)
    o = _opts(tol, maxit, prec, max_refine, check_every, inner_tol)
    code = lib().nys_pcg_solve_ragged(cops, cps, mu_arr, barr, xarr, npb, ctypes.byref(o), ctypes.byref(info),
                                      _ptr(ws), ws.numel(), _stream())
    _check(code, allow_not_converged=True)
    return Xs, SolveInfo(list(it), list(rr), list(st), info.refine_steps, info.total_iters, code)


def nys_pcg_solve_ragged_device(ops: Sequence[Operator], Ps: Sequence[Precond], mus: Sequence[float],
                                Bs: Sequence[torch.Tensor], Xs: Sequence[torch.Tensor], iters: torch.Tensor,
                                relres: torch.Tensor, status: torch.Tensor, tol: float = 1e-10, maxit: int = 500,
                                prec: int = NYS_PREC_FP64, max_refine: int = 10, inner_tol: float = 1e-4,
                                ws: Optional[torch.Tensor] = None):
    """Device-info form of nys_pcg_solve_ragged (opts.device_info = 1): no host
    synchronisation, so it can be captured into a graph.  Bs, Xs: contiguous
    float64 device vectors (Xs: in x0, out x); iters / relres / status: device
    tensors of len(ops) entries written by the call's last kernels.  Runs
    exactly maxit iterations per step (float64: one step; refinement modes:
    max_refine steps).  Returns (refine_steps, total_iters)."""
    npb = len(ops)
    for v in list(Bs) + list(Xs):
        if v.dtype != torch.float64 or not v.is_contiguous() or not v.is_cuda:
            raise ValueError("Bs and Xs must be contiguous float64 device vectors")
    for t, dt in ((iters, torch.int32), (relres, torch.float64), (status, torch.int32)):
        if t.dtype != dt or t.numel() < npb or not t.is_cuda:
            raise ValueError("iters / relres / status: device tensors of int32 / float64 / int32, %d entries" % npb)
    cops = (_Operator * npb)(*[o.c() for o in ops])
    cps = (_Precond * npb)(*[p.c() for p in Ps])
    mu_arr = (ctypes.c_double * npb)(*[float(m) for m in mus])
    barr = (ctypes.c_void_p * npb)(*[_ptr(b) for b in Bs])
    xarr = (ctypes.c_void_p * npb)(*[_ptr(x) for x in Xs])
    if ws is None:
        nb = lib().nys_workspace_size_ragged(cops, cps, npb, prec)
        ws = torch.empty(nb, dtype=torch.uint8, device=Bs[0].device)
    info = _Info(ctypes.cast(ctypes.c_void_p(iters.data_ptr()), ctypes.POINTER(ctypes.c_int32)),
                 ctypes.cast(ctypes.c_void_p(relres.data_ptr()), ctypes.POINTER(ctypes.c_double)),
                 ctypes.cast(ctypes.c_void_p(status.data_ptr()), ctypes.POINTER(ctypes.c_int32)), 0, 0)
    o = _opts(tol, maxit, prec, max_refine, 1, inner_tol, device_info=1)
    _check(lib().nys_pcg_solve_ragged(cops, cps, mu_arr, barr, xarr, npb, ctypes.byref(o), ctypes.byref(info),
                                      _ptr(ws), ws.numel(), _stream()))
    return info.refine_steps, info.total_iters


def nys_pcg_backward(op: Operator, P: Precond, mu: float, x: torch.Tensor, gx: torch.Tensor,
                     want_sigma: bool = False, want_X: bool = False, tol: float = 1e-10, maxit: int = 500,
                     prec: int = NYS_PREC_FP64, max_refine: int = 10, check_every: int = 0,
                     inner_tol: float = 1e-4, ws: Optional[torch.Tensor] = None,
                     raise_on_not_converged: bool = False):
    """Adjoint solve with the same preconditioner.  Returns dict(gb, gmu, gsigma, gX, info)."""
    x = x.reshape(-1).contiguous().to(torch.float64)
    gx = gx.reshape(-1).contiguous().to(torch.float64)
    gb = torch.zeros_like(x)
    gX = torch.empty(op.data.shape[0], op.n, dtype=torch.float64, device=x.device) if want_X else None
    gmu = ctypes.c_double(0.0)
    gsig = ctypes.c_double(0.0)
    w = _ws(op, P.U.shape[1], 1, prec, ws)
    it = (ctypes.c_int32 * 1)()
    rr = (ctypes.c_double * 1)()
    st = (ctypes.c_int32 * 1)()
    info = _Info(it, rr, st, 0, 0)
    o = _opts(tol, maxit, prec, max_refine, check_every, inner_tol)
    code = lib().nys_pcg_backward(ctypes.byref(op.c()), ctypes.byref(P.c()), float(mu), _ptr(x), _ptr(gx),
                                  _ptr(gb), ctypes.byref(gmu), ctypes.byref(gsig) if want_sigma else None,
                                  _ptr(gX), ctypes.byref(o), ctypes.byref(info), _ptr(w), w.numel(), _stream())
    _check(code, allow_not_converged=not raise_on_not_converged)
    return dict(gb=gb, gmu=gmu.value, gsigma=gsig.value if want_sigma else None, gX=gX,
                info=SolveInfo(list(it), list(rr), list(st), info.refine_steps, info.total_iters, code))


def nys_rbf_cross(op: Operator, Xv: torch.Tensor, v: torch.Tensor, transpose: bool = False,
                  wvec: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """K(Xv, X) v (transpose=False, v: n), K(Xv, X)^T v (transpose=True, v: nv), or with
    wvec (n): (out, v^T out) for out = (dK(Xv, X)/dsigma) wvec and v of length nv."""
    Xv = Xv.contiguous()
    v = v.reshape(-1).contiguous().to(torch.float64)
    nv = Xv.shape[0]
    want = nv if (transpose or wvec is not None) else op.n
    if v.numel() != want:
        raise ValueError("nys_rbf_cross: v has %d entries, expected %d" % (v.numel(), want))
    if wvec is not None and (transpose or wvec.numel() != op.n):
        raise ValueError("nys_rbf_cross: wvec needs n = %d entries and transpose=False" % op.n)
    out = torch.empty(op.n if transpose else nv, dtype=torch.float64, device=v.device)
    dsig = ctypes.c_double(0.0)
    if ws is None:
        ws = torch.empty(8 * 1024 * max(op.n, nv) + 8192, dtype=torch.uint8, device=v.device)
    wv = None if wvec is None else wvec.reshape(-1).contiguous().to(torch.float64)
    _check(lib().nys_rbf_cross(ctypes.byref(op.c()), _ptr(Xv), nv, Xv.stride(0), 1 if transpose else 0, _ptr(v),
                               _ptr(out), _ptr(wv), ctypes.byref(dsig) if wv is not None else None, _ptr(ws),
                               ws.numel(), _stream()))
    return (out, dsig.value) if wv is not None else out


from .autograd import NystromSolve, RbfCross, nystrom_solve, rbf_cross  # noqa: E402,F401
