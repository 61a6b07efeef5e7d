"""Thin ctypes binding of librbcg.so (C ABI in include/rbcg.h).

Only argument marshalling happens here: every step of the solvers runs in the
library's HIP kernels.  PyTorch provides device memory and the stream.  If the
compiled library is missing, importing this module raises ImportError: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbcg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"librbcg.so not built ({LIB_PATH}); run `python -m paper_2501_18717_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "NOT_SPD", -3: "BREAKDOWN", -4: "NO_CONVERGENCE",
          -5: "HIP", -6: "OOM", -7: "UNSUPPORTED", -8: "TOO_LARGE"}


class Opts(ctypes.Structure):
    _fields_ = [("t_max", ctypes.c_int32), ("rtol", ctypes.c_double), ("matvec", ctypes.c_int32),
                ("refine_max", ctypes.c_int32), ("nquad", ctypes.c_int32), ("group", ctypes.c_int32),
                ("eta", ctypes.c_double), ("sweep_tol", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("reorth", ctypes.c_int32), ("reorth_blocks", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("matrix_loads", ctypes.c_int32),
                ("refine_sweeps", ctypes.c_int32), ("deflated", ctypes.c_int32),
                ("precision_used", ctypes.c_int32), ("relres", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_status_string = _sig("rbcg_status_string", ctypes.c_char_p, [ctypes.c_int])
_version = _sig("rbcg_version", ctypes.c_int, [])
_create = _sig("rbcg_create", ctypes.c_int, [ctypes.POINTER(_vp), _vp])
_destroy = _sig("rbcg_destroy", ctypes.c_int, [_vp])
_op_dense = _sig("rbcg_op_create_dense", ctypes.c_int, [_vp, ctypes.POINTER(_vp), _i64, _vp, _i64, ctypes.c_int])
_op_dense_host = _sig("rbcg_op_create_dense_host", ctypes.c_int,
                      [_vp, ctypes.POINTER(_vp), _i64, _vp, _i64, _i64, ctypes.c_int])
_op_gram = _sig("rbcg_op_create_gram", ctypes.c_int, [_vp, ctypes.POINTER(_vp), _i64, _i64, _vp, _i64, ctypes.c_int])
_op_destroy = _sig("rbcg_op_destroy", ctypes.c_int, [_vp])
_solve = _sig("rbcg_solve", ctypes.c_int, [_vp, _i64, ctypes.POINTER(_vp), _dp, ctypes.POINTER(_vp),
                                            ctypes.POINTER(_vp), ctypes.POINTER(_i32), ctypes.POINTER(_vp),
                                            ctypes.POINTER(Opts), ctypes.POINTER(Info)])
_path = _sig("rbcg_path", ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i64, _dp, _vp, ctypes.POINTER(Opts),
                                          ctypes.POINTER(Info)])
_sqrt = _sig("rbcg_sqrt_apply", ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)])
_invsqrt = _sig("rbcg_invsqrt_apply", ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)])
_ws_bytes = _sig("rbcg_workspace_bytes", _i64, [_vp])
_op_apply = _sig("rbcg_op_apply", ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, ctypes.c_int])
_op_apply_noalloc = _sig("rbcg_op_apply_noalloc", ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, ctypes.c_int])
_omega_fill = _sig("rbcg_omega_fill", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint32, _i64, _i64, _vp, _i64])
_nystrom_pcg = _sig("rbcg_nystrom_pcg", ctypes.c_int,
                    [_vp, _vp, _vp, _vp, _i32, _i32, ctypes.c_double, ctypes.c_double, _vp, ctypes.POINTER(Opts),
                     ctypes.POINTER(Info), _dp, ctypes.POINTER(_i32), _dp])
_noalloc_bytes = _sig("rbcg_noalloc_scratch_bytes", _i64, [])
_sqrt_rule = _sig("rbcg_sqrt_rule", ctypes.c_int, [ctypes.c_double, ctypes.c_double, _i32, _dp, _dp])
_profile = _sig("rbcg_profile", ctypes.c_int, [_vp, ctypes.c_int])
_profile_read = _sig("rbcg_profile_read", ctypes.c_int, [_vp, ctypes.POINTER(_i64), _dp, _dp, _dp])


class RbcgError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({_status_string(code).decode()})")
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise RbcgError(code, where)


def status_string(code: int) -> str:
    return _status_string(code).decode()


def version() -> int:
    return _version()


def sqrt_rule(lo: float, hi: float, n: int):
    """Host-only quadrature rule of the square-root integral (shifts, weights)."""
    s = (ctypes.c_double * n)()
    w = (ctypes.c_double * n)()
    _check(_sqrt_rule(lo, hi, n, s, w), "rbcg_sqrt_rule")
    return list(s), list(w)


def _ptr(t) -> int:
    return t.data_ptr()


def _need(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


REORTH = {"full": 0, "none": 1, "partial": 2}


def opts(t_max: int, rtol: float = 0.0, matvec: str = "f64", refine_max: int = 1, nquad: int = 0, group: int = 0,
         eta: float = 0.0, sweep_tol: float = 0.0, seed: int = 0, reorth: str = "full", reorth_blocks: int = 0) -> Opts:
    return Opts(int(t_max), float(rtol), DTYPES[matvec], int(refine_max), int(nquad), int(group), float(eta),
                float(sweep_tol), int(seed) & 0xFFFFFFFFFFFFFFFF, REORTH[reorth], int(reorth_blocks))


class Context:
    """Binds a HIP stream (torch's current stream by default) and owns the workspace."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _vp()
        _check(_create(ctypes.byref(h), _vp(stream.cuda_stream)), "rbcg_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self) -> int:
        return int(_ws_bytes(self._h))

    def profile(self, enable: bool, every: int = 1):
        """Start (clearing counters) or stop event timing of every `every`-th block-product GEMM."""
        if enable and every < 1:
            raise ValueError("every must be >= 1")
        _check(_profile(self._h, int(every) if enable else 0), "rbcg_profile")

    def profile_read(self) -> dict:
        n = _i64()
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)),
               "rbcg_profile_read")
        return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}

    def close(self):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DenseOperator:
    """A (d x d, FP64, symmetric) with an optional FP32 copy for mixed-precision products."""

    def __init__(self, ctx: Context, A, lo: str = "f64"):
        import torch
        _need(A, torch.float64, name="A")
        d = A.shape[0]
        if A.dim() != 2 or A.shape[1] != d:
            raise ValueError("A must be square")
        h = _vp()
        _check(_op_dense(ctx.handle, ctypes.byref(h), d, _ptr(A), d, DTYPES[lo]), "rbcg_op_create_dense")
        self._h, self.A, self.d, self.ctx = h, A, d, ctx

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DenseHostOperator(DenseOperator):
    """A (d x d, FP64, symmetric) kept in page-locked host memory; every product streams it to
    the GPU in chunks of `chunk_rows` rows.  lo="f32" also keeps a pinned FP32 copy on the host,
    which FP32 products stream."""

    def __init__(self, ctx: Context, A, chunk_rows: int, lo: str = "f64"):
        import torch
        if not isinstance(A, torch.Tensor) or A.is_cuda or A.dtype != torch.float64 or not A.is_contiguous():
            raise ValueError("A must be a contiguous FP64 CPU tensor")
        if not A.is_pinned():
            raise ValueError("A must be in page-locked memory (pin_memory=True)")
        d = A.shape[0]
        if A.dim() != 2 or A.shape[1] != d:
            raise ValueError("A must be square")
        h = _vp()
        _check(_op_dense_host(ctx.handle, ctypes.byref(h), d, _ptr(A), d, int(chunk_rows), DTYPES[lo]),
               "rbcg_op_create_dense_host")
        self._h, self.A, self.d, self.ctx = h, A, d, ctx


class GramOperator:
    """A = Z^T Z with Z (n x d, FP32) and optional BF16 copies of Z and Z^T."""

    def __init__(self, ctx: Context, Z, lo: str = "f64"):
        import torch
        _need(Z, torch.float32, name="Z")
        n, d = Z.shape
        h = _vp()
        _check(_op_gram(ctx.handle, ctypes.byref(h), n, d, _ptr(Z), d, DTYPES[lo]), "rbcg_op_create_gram")
        self._h, self.Z, self.n, self.d, self.ctx = h, Z, n, d, ctx

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def op_apply(ctx: Context, op, X, W, matvec: str = "f64"):
    """W = A X (rows of X) with the solvers' block product in the given precision."""
    import torch
    N, d = X.shape
    _need(X, torch.float64, (N, op.d), "X")
    _need(W, torch.float64, (N, op.d), "W")
    _check(_op_apply(ctx.handle, op.handle, N, _ptr(X), _ptr(W), DTYPES[matvec]), "rbcg_op_apply")


def op_apply_noalloc(ctx: Context, op, X, W, matvec: str = "f64"):
    """The same product through rbcg_op_apply_noalloc (fixed per-GPU scratch, no allocation)."""
    import torch
    N, d = X.shape
    _need(X, torch.float64, (N, op.d), "X")
    _need(W, torch.float64, (N, op.d), "W")
    _check(_op_apply_noalloc(ctx.handle, op.handle, N, _ptr(X), _ptr(W), DTYPES[matvec]), "rbcg_op_apply_noalloc")


def omega_fill(ctx: Context, seed: int, stream: int, out):
    """rbcg_omega_fill: out (rows x cols FP64 device tensor) = the seeded Gaussian block."""
    import torch
    if not out.is_cuda or out.dtype != torch.float64 or out.dim() != 2 or out.stride(1) != 1:
        raise ValueError("out must be a 2-D FP64 device tensor with unit column stride")
    rows, cols = out.shape
    _check(_omega_fill(ctx.handle, ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), ctypes.c_uint32(int(stream)),
                       rows, cols, _ptr(out), out.stride(0)), "rbcg_omega_fill")


def nystrom_pcg(ctx: Context, op, b, omega, s: int, mu: float, x, options: Opts, theta: float = 0.0,
                check: bool = True):
    """rbcg_nystrom_pcg: x written in place.  `omega` is a (k, d) tensor or an int k (drawn from
    options.seed).  Returns (rc, info, eigenvalues (descending, s k values), rank, theta)."""
    import torch
    d = op.d
    _need(b, torch.float64, (d,), "b")
    _need(x, torch.float64, (d,), "x")
    if isinstance(omega, int):
        k, om = omega, None
    else:
        _need(omega, torch.float64, name="omega")
        if omega.dim() != 2 or omega.shape[1] != d:
            raise ValueError("omega must have shape (k, d)")
        k, om = omega.shape[0], _ptr(omega)
    r = max(1, s * k)
    eig = (ctypes.c_double * r)()
    rank = _i32()
    th = ctypes.c_double()
    info = Info()
    rc = _nystrom_pcg(ctx.handle, op.handle, _ptr(b), om, k, s, float(mu), float(theta), _ptr(x),
                      ctypes.byref(options), ctypes.byref(info), eig, ctypes.byref(rank), ctypes.byref(th))
    if check and rc not in (0, -4):
        raise RbcgError(rc, "rbcg_nystrom_pcg")
    return rc, info.as_dict(), list(eig)[: s * k], rank.value, th.value


def noalloc_scratch_bytes() -> int:
    return int(_noalloc_bytes())


def solve(ctx: Context, ops: Sequence, mus: Sequence[float], bs: Sequence, omegas: Sequence, xs: Sequence,
          options: Sequence[Opts], check: bool = True):
    """rbcg_solve over len(ops) independent systems; x tensors are written in place.  An entry of
    `omegas` is a (k, d) tensor, None (k = 0), or an int k: a k x d block drawn on the device from
    that system's options.seed."""
    import torch
    n = len(ops)
    assert len(mus) == n and len(bs) == n and len(omegas) == n and len(xs) == n and len(options) == n
    ks = []
    for i in range(n):
        d = ops[i].d
        _need(bs[i], torch.float64, (d,), "b")
        _need(xs[i], torch.float64, (d,), "x")
        om = omegas[i]
        if isinstance(om, int):
            ks.append(om)
        elif om is not None and om.numel():
            _need(om, torch.float64, name="omega")
            if om.dim() != 2 or om.shape[1] != d:
                raise ValueError("omega must have shape (k, d)")
            ks.append(om.shape[0])
        else:
            ks.append(0)
    op_arr = (_vp * n)(*[o.handle for o in ops])
    mu_arr = (ctypes.c_double * n)(*[float(m) for m in mus])
    b_arr = (_vp * n)(*[_ptr(b) for b in bs])
    om_arr = (_vp * n)(*[(_ptr(o) if (o is not None and not isinstance(o, int) and o.numel()) else None)
                         for o in omegas])
    k_arr = (_i32 * n)(*ks)
    x_arr = (_vp * n)(*[_ptr(x) for x in xs])
    o_arr = (Opts * n)(*options)
    info = (Info * n)()
    rc = _solve(ctx.handle, n, op_arr, mu_arr, b_arr, om_arr, k_arr, x_arr, o_arr, info)
    infos = [i.as_dict() for i in info]
    if check and rc not in (0, -4):
        raise RbcgError(rc, "rbcg_solve")
    return rc, infos


def path(ctx: Context, op, b, omega, mus: Sequence[float], X, options: Opts, check: bool = True):
    """rbcg_path: X (L x d) written in place.  `omega` is a (k, d) tensor, None (k = 0), or an int
    k: a k x d block drawn on the device from options.seed."""
    import torch
    d = op.d
    L = len(mus)
    _need(b, torch.float64, (d,), "b")
    _need(X, torch.float64, (L, d), "X")
    k = 0
    seeded = isinstance(omega, int)
    if seeded:
        k = omega
    elif omega is not None and omega.numel():
        _need(omega, torch.float64, name="omega")
        k = omega.shape[0]
    mu_arr = (ctypes.c_double * L)(*[float(m) for m in mus])
    info = (Info * L)()
    rc = _path(ctx.handle, op.handle, _ptr(b), _ptr(omega) if (k and not seeded) else None, k, L, mu_arr, _ptr(X),
               ctypes.byref(options), info)
    infos = [i.as_dict() for i in info]
    if check and rc not in (0, -4):
        raise RbcgError(rc, "rbcg_path")
    return rc, infos


def _sqrt_call(fn, name, ctx, op, B, Y, options, check):
    import torch
    ms, d = B.shape
    _need(B, torch.float64, (ms, op.d), "B")
    _need(Y, torch.float64, (ms, op.d), "Y")
    info = (Info * ms)()
    rc = fn(ctx.handle, op.handle, ms, _ptr(B), _ptr(Y), ctypes.byref(options), info)
    infos = [i.as_dict() for i in info]
    if check and rc != 0:
        raise RbcgError(rc, name)
    return rc, infos


def sqrt_apply(ctx: Context, op, B, Y, options: Opts, check: bool = True):
    """rbcg_sqrt_apply: Y (m_s x d) ~ rows of A^(1/2) B^T, written in place."""
    return _sqrt_call(_sqrt, "rbcg_sqrt_apply", ctx, op, B, Y, options, check)


def invsqrt_apply(ctx: Context, op, B, Y, options: Opts, check: bool = True):
    """rbcg_invsqrt_apply: Y (m_s x d) ~ rows of A^(-1/2) B^T, written in place."""
    return _sqrt_call(_invsqrt, "rbcg_invsqrt_apply", ctx, op, B, Y, options, check)
