"""Python binding of libpk: argument marshalling only.

Tensors are torch CUDA (HIP) float32 tensors; every computation runs in the
library's gfx950 kernels.  Calls are asynchronous on the current torch stream
(or the ``stream`` given).  Errors from the library raise ``PkError``; type,
device and layout problems raise ``TypeError``/``ValueError`` before the call.
"""
from __future__ import annotations

import ctypes
from contextlib import contextmanager

import torch

from . import _lib

PRECISIONS = {"fp32": 0, "bf16": 1, "split": 2, "split_bf16": 2}
KERNELS = {"gemm": 0, "gemm3": 1, "gemv": 2, "gemv_t": 3, "gemv_pair": 4, "conv2d": 5,
           "conv3d": 6, "colstats": 7, "corr": 8, "convert": 9, "covar": 10, "syrk": 11,
           "syr2k": 12, "gesummv": 13, "mvt": 14, "fdtd2d": 15}
FAMILY_IDS = {"gemm_f32": 0, "gemm_bf16": 1, "gemm_split": 2, "gemv": 3, "gemv_t": 4,
              "gemv_pair": 5, "conv2d": 6, "conv3d": 7, "colstats": 8, "syrk_f32": 9,
              "syrk_bf16": 10, "syrk_split": 11, "convert": 12, "rankk": 13, "gesummv": 14,
              "fdtd": 15, "gemm_bf16_ws": 16, "gemm_split_ws": 17}


class PkError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"pk status {status}: {message}")


def _check(status: int):
    if status != 0:
        lib = _lib.load()
        detail = lib.pk_last_error().decode(errors="replace")
        name = lib.pk_status_string(status).decode()
        raise PkError(status, f"{name}: {detail}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _f32(t, name, dims=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if dims is not None and t.dim() != dims:
        raise ValueError(f"{name} must be {dims}-D, got shape {tuple(t.shape)}")
    return t


def _rows(t, name):
    """Row-major 2-D view with unit column stride; returns the row stride."""
    _f32(t, name, 2)
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError(f"{name} must have unit column stride")
    return max(t.stride(0), t.shape[1], 1)


def _vec(t, name, n):
    _f32(t, name, 1)
    if t.shape[0] != n:
        raise ValueError(f"{name} must have {n} entries, got {t.shape[0]}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """One libpk context (device, loaded code objects, variant table)."""

    def __init__(self, device: int | None = None):
        lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib.pk_context_create(self.device, ctypes.byref(h)))
        self.handle = h
        self._lib = lib

    def close(self):
        if self.handle:
            self._lib.pk_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_checks(self, enabled: bool):
        _check(self._lib.pk_context_set_checks(self.handle, int(bool(enabled))))

    # -- workspace -------------------------------------------------------------------
    @staticmethod
    def workspace_bytes(kernel: str, dims, prec: str = "fp32") -> int:
        lib = _lib.load()
        arr = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
        out = ctypes.c_size_t()
        _check(lib.pk_workspace_bytes(KERNELS[kernel], arr, len(dims), PRECISIONS[prec],
                                      ctypes.byref(out)))
        return int(out.value)

    def _ws(self, ws, kernel, dims, prec="fp32", device=None):
        need = self.workspace_bytes(kernel, dims, prec)
        if ws is None:
            if need == 0:
                return None, 0
            ws = torch.empty(need, dtype=torch.uint8, device=device or f"cuda:{self.device}")
        nbytes = ws.numel() * ws.element_size()
        return ws, nbytes

    # -- kernels ----------------------------------------------------------------------
    def gemm(self, A, B, C, alpha=1.0, beta=0.0, prec="fp32", ws=None, stream=None):
        """C <- alpha * A @ B + beta * C (in place); returns C.

        For bf16 / split the operands are prepared once in a workspace
        (pk_sgemm_ws; `ws` a uint8 tensor, allocated here when None); `ws=False`
        uses the kernel that rounds the operands inside its main loop (pk_sgemm)."""
        lda, ldb, ldc = _rows(A, "A"), _rows(B, "B"), _rows(C, "C")
        M, K = A.shape
        K2, N = B.shape
        if K2 != K or tuple(C.shape) != (M, N):
            raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
        if prec == "fp32" or ws is False:
            _check(self._lib.pk_sgemm(self.handle, PRECISIONS[prec], M, N, K, float(alpha), _ptr(A), lda,
                                      _ptr(B), ldb, float(beta), _ptr(C), ldc, _stream(stream)))
            return C
        ws, nb = self._ws(ws, "gemm", (M, N, K), prec, A.device)
        _check(self._lib.pk_sgemm_ws(self.handle, PRECISIONS[prec], M, N, K, float(alpha), _ptr(A), lda,
                                     _ptr(B), ldb, float(beta), _ptr(C), ldc, _ptr(ws), nb, _stream(stream)))
        return C

    def gemm3(self, A, B, Cm, D, alpha=1.0, beta=0.0, prec="fp32", ws=None, stream=None):
        """D <- alpha * (A @ B) @ Cm + beta * D (in place); returns D."""
        lda, ldb, ldc, ldd = _rows(A, "A"), _rows(B, "B"), _rows(Cm, "Cm"), _rows(D, "D")
        M, K = A.shape
        K2, L = B.shape
        L2, N = Cm.shape
        if K2 != K or L2 != L or tuple(D.shape) != (M, N):
            raise ValueError("shape mismatch in gemm3")
        ws, nb = self._ws(ws, "gemm3", (M, N, K, L), prec, A.device)
        _check(self._lib.pk_sgemm3(self.handle, PRECISIONS[prec], M, N, K, L, float(alpha), _ptr(A), lda,
                                   _ptr(B), ldb, _ptr(Cm), ldc, float(beta), _ptr(D), ldd, _ptr(ws), nb,
                                   _stream(stream)))
        return D

    def gemv(self, A, x, y=None, stream=None):
        """y = A @ x."""
        lda = _rows(A, "A")
        M, N = A.shape
        _vec(x, "x", N)
        if y is None:
            y = torch.empty(M, dtype=torch.float32, device=A.device)
        _vec(y, "y", M)
        _check(self._lib.pk_sgemv(self.handle, M, N, _ptr(A), lda, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def gemv_t(self, A, z, y=None, ws=None, stream=None):
        """y = A.T @ z."""
        lda = _rows(A, "A")
        M, N = A.shape
        _vec(z, "z", M)
        if y is None:
            y = torch.empty(N, dtype=torch.float32, device=A.device)
        _vec(y, "y", N)
        ws, nb = self._ws(ws, "gemv_t", (M, N), device=A.device)
        _check(self._lib.pk_sgemv_t(self.handle, M, N, _ptr(A), lda, _ptr(z), _ptr(y), _ptr(ws), nb,
                                    _stream(stream)))
        return y

    def gemv_pair(self, A, x, z, y1=None, y2=None, ws=None, stream=None):
        """(A @ x, A.T @ z) in one pass over A."""
        lda = _rows(A, "A")
        M, N = A.shape
        _vec(x, "x", N)
        _vec(z, "z", M)
        if y1 is None:
            y1 = torch.empty(M, dtype=torch.float32, device=A.device)
        if y2 is None:
            y2 = torch.empty(N, dtype=torch.float32, device=A.device)
        _vec(y1, "y1", M)
        _vec(y2, "y2", N)
        ws, nb = self._ws(ws, "gemv_pair", (M, N), device=A.device)
        _check(self._lib.pk_sgemv_pair(self.handle, M, N, _ptr(A), lda, _ptr(x), _ptr(z), _ptr(y1),
                                       _ptr(y2), _ptr(ws), nb, _stream(stream)))
        return y1, y2

    def conv2d(self, grid, taps, out=None, stream=None):
        """3x3 stencil (no flip), zero border."""
        ldi = _rows(grid, "grid")
        H, W = grid.shape
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=grid.device)
        ldo = _rows(out, "out")
        if tuple(out.shape) != (H, W):
            raise ValueError("out shape mismatch")
        w = (ctypes.c_float * 9)(*[float(v) for v in torch.as_tensor(taps).reshape(-1).tolist()])
        _check(self._lib.pk_conv2d_3x3(self.handle, H, W, w, _ptr(grid), ldi, _ptr(out), ldo,
                                       _stream(stream)))
        return out

    def conv3d(self, vol, taps, out=None, stream=None):
        """3x3x3 stencil (no flip) on a contiguous D x H x W volume, zero faces."""
        _f32(vol, "vol", 3)
        if not vol.is_contiguous():
            raise ValueError("vol must be contiguous")
        D, H, W = vol.shape
        if out is None:
            out = torch.empty_like(vol)
        _f32(out, "out", 3)
        if tuple(out.shape) != (D, H, W) or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of the same shape")
        tl = torch.as_tensor(taps).reshape(-1).tolist()
        if len(tl) != 27:
            raise ValueError("conv3d needs 27 taps")
        w = (ctypes.c_float * 27)(*[float(v) for v in tl])
        _check(self._lib.pk_conv3d_3x3x3(self.handle, D, H, W, w, _ptr(vol), _ptr(out), _stream(stream)))
        return out

    def colstats(self, X, eps, mean=None, std=None, ws=None, stream=None):
        """Column mean and deviation (n-1), floored at eps."""
        ldx = _rows(X, "X")
        n, m = X.shape
        if mean is None:
            mean = torch.empty(m, dtype=torch.float32, device=X.device)
        if std is None:
            std = torch.empty(m, dtype=torch.float32, device=X.device)
        _vec(mean, "mean", m)
        _vec(std, "std", m)
        ws, nb = self._ws(ws, "colstats", (n, m), device=X.device)
        _check(self._lib.pk_colstats(self.handle, n, m, _ptr(X), ldx, float(eps), _ptr(mean), _ptr(std),
                                     _ptr(ws), nb, _stream(stream)))
        return mean, std

    def corr(self, X, eps, prec="fp32", R=None, mean=None, std=None, ws=None, stream=None):
        """Correlation matrix of the columns of X; returns (R, mean, std)."""
        ldx = _rows(X, "X")
        n, m = X.shape
        if R is None:
            R = torch.empty((m, m), dtype=torch.float32, device=X.device)
        ldr = _rows(R, "R")
        if tuple(R.shape) != (m, m):
            raise ValueError("R must be m x m")
        if mean is None:
            mean = torch.empty(m, dtype=torch.float32, device=X.device)
        if std is None:
            std = torch.empty(m, dtype=torch.float32, device=X.device)
        _vec(mean, "mean", m)
        _vec(std, "std", m)
        ws, nb = self._ws(ws, "corr", (n, m), prec, X.device)
        _check(self._lib.pk_corr(self.handle, PRECISIONS[prec], n, m, _ptr(X), ldx, float(eps), _ptr(mean),
                                 _ptr(std), _ptr(R), ldr, _ptr(ws), nb, _stream(stream)))
        return R, mean, std

    def corr_noalloc(self, X, eps, R, mean, std, prec="fp32", stream=None):
        """pk_corr_noalloc: the correlation into the caller's R, mean and std with the
        library's static scratch as workspace (nothing is allocated, here or below)."""
        ldx = _rows(X, "X")
        n, m = X.shape
        ldr = _rows(R, "R")
        if tuple(R.shape) != (m, m):
            raise ValueError("R must be m x m")
        _vec(mean, "mean", m)
        _vec(std, "std", m)
        _check(self._lib.pk_corr_noalloc(self.handle, PRECISIONS[prec], n, m, _ptr(X), ldx, float(eps),
                                         _ptr(mean), _ptr(std), _ptr(R), ldr, _stream(stream)))
        return R, mean, std

    def covar(self, X, prec="fp32", C=None, mean=None, ws=None, stream=None):
        """Covariance matrix of the columns of X; returns (C, mean)."""
        ldx = _rows(X, "X")
        n, m = X.shape
        if C is None:
            C = torch.empty((m, m), dtype=torch.float32, device=X.device)
        ldc = _rows(C, "C")
        if tuple(C.shape) != (m, m):
            raise ValueError("C must be m x m")
        if mean is None:
            mean = torch.empty(m, dtype=torch.float32, device=X.device)
        _vec(mean, "mean", m)
        ws, nb = self._ws(ws, "covar", (n, m), prec, X.device)
        _check(self._lib.pk_covar(self.handle, PRECISIONS[prec], n, m, _ptr(X), ldx, _ptr(mean), _ptr(C), ldc,
                                  _ptr(ws), nb, _stream(stream)))
        return C, mean

    def syrk(self, A, C, alpha=1.0, beta=0.0, stream=None):
        """C <- alpha A A^T + beta C (in place); returns C."""
        lda, ldc = _rows(A, "A"), _rows(C, "C")
        N, K = A.shape
        if tuple(C.shape) != (N, N):
            raise ValueError("C must be N x N")
        _check(self._lib.pk_ssyrk(self.handle, N, K, float(alpha), _ptr(A), lda, float(beta), _ptr(C), ldc,
                                  _stream(stream)))
        return C

    def syr2k(self, A, B, C, alpha=1.0, beta=0.0, stream=None):
        """C <- alpha (A B^T + B A^T) + beta C (in place); returns C."""
        lda, ldb, ldc = _rows(A, "A"), _rows(B, "B"), _rows(C, "C")
        N, K = A.shape
        if tuple(B.shape) != (N, K) or tuple(C.shape) != (N, N):
            raise ValueError("shape mismatch in syr2k")
        _check(self._lib.pk_ssyr2k(self.handle, N, K, float(alpha), _ptr(A), lda, _ptr(B), ldb, float(beta),
                                   _ptr(C), ldc, _stream(stream)))
        return C

    def gesummv(self, A, B, x, alpha=1.0, beta=1.0, y=None, stream=None):
        """alpha A x + beta B x."""
        lda, ldb = _rows(A, "A"), _rows(B, "B")
        N = A.shape[0]
        if tuple(A.shape) != (N, N) or tuple(B.shape) != (N, N):
            raise ValueError("A and B must be N x N")
        _vec(x, "x", N)
        if y is None:
            y = torch.empty(N, dtype=torch.float32, device=A.device)
        _vec(y, "y", N)
        _check(self._lib.pk_sgesummv(self.handle, N, float(alpha), _ptr(A), lda, float(beta), _ptr(B), ldb,
                                     _ptr(x), _ptr(y), _stream(stream)))
        return y

    def mvt(self, A, y1, y2, x1, x2, ws=None, stream=None):
        """x1 += A y1 and x2 += A^T y2 (in place, one pass over A); returns (x1, x2)."""
        lda = _rows(A, "A")
        N = A.shape[0]
        if tuple(A.shape) != (N, N):
            raise ValueError("A must be N x N")
        for t, nm in ((y1, "y1"), (y2, "y2"), (x1, "x1"), (x2, "x2")):
            _vec(t, nm, N)
        ws, nb = self._ws(ws, "mvt", (N,), device=A.device)
        _check(self._lib.pk_smvt(self.handle, N, _ptr(A), lda, _ptr(y1), _ptr(y2), _ptr(x1), _ptr(x2),
                                 _ptr(ws), nb, _stream(stream)))
        return x1, x2

    def fdtd2d(self, fict, ex, ey, hz, stream=None):
        """len(fict) FDTD-2D steps on ex, ey, hz (updated in place); returns (ex, ey, hz)."""
        _f32(fict, "fict", 1)
        for t, nm in ((ex, "ex"), (ey, "ey"), (hz, "hz")):
            _f32(t, nm, 2)
            if not t.is_contiguous() or tuple(t.shape) != tuple(ex.shape):
                raise ValueError(f"{nm} must be contiguous and match ex")
        NX, NY = ex.shape
        _check(self._lib.pk_fdtd2d(self.handle, fict.numel(), NX, NY, _ptr(fict), _ptr(ex), _ptr(ey), _ptr(hz),
                                   _stream(stream)))
        return ex, ey, hz

    def convert_bf16(self, x, split=False, stream=None):
        """bfloat16 bits (int16 tensors) of x: hi, or (hi, lo) when split."""
        _f32(x, "x")
        if not x.is_contiguous():
            raise ValueError("x must be contiguous")
        n = x.numel()
        hi = torch.empty(x.shape, dtype=torch.int16, device=x.device)
        lo = torch.empty(x.shape, dtype=torch.int16, device=x.device) if split else None
        _check(self._lib.pk_convert_bf16(self.handle, n, _ptr(x), _ptr(hi), _ptr(lo), _stream(stream)))
        return (hi, lo) if split else hi

    # -- variants ---------------------------------------------------------------------------
    def variant_load(self, code: bytes) -> int:
        out = ctypes.c_int32(-1)
        _check(self._lib.pk_variant_load(self.handle, code, len(code), ctypes.byref(out)))
        return int(out.value)

    def variant_unload(self, vid: int):
        _check(self._lib.pk_variant_unload(self.handle, int(vid)))

    def variant_info(self, vid: int):
        fam = ctypes.c_int32()
        knobs = (ctypes.c_int32 * 16)()
        h = ctypes.c_uint64()
        _check(self._lib.pk_variant_info(self.handle, int(vid), ctypes.byref(fam), knobs, ctypes.byref(h)))
        return int(fam.value), list(knobs), int(h.value)

    def variant_default(self, family) -> int:
        fid = FAMILY_IDS[family] if isinstance(family, str) else int(family)
        out = ctypes.c_int32(-1)
        _check(self._lib.pk_variant_default(self.handle, fid, ctypes.byref(out)))
        return int(out.value)

    def variant_select(self, family, vid: int):
        fid = FAMILY_IDS[family] if isinstance(family, str) else int(family)
        _check(self._lib.pk_variant_select(self.handle, fid, int(vid)))

    def variant_set_best(self, family, bucket: int, vid: int):
        fid = FAMILY_IDS[family] if isinstance(family, str) else int(family)
        _check(self._lib.pk_variant_set_best(self.handle, fid, int(bucket), int(vid)))

    @staticmethod
    def size_bucket(d: int) -> int:
        return int(_lib.load().pk_size_bucket(int(d)))

    # -- graphs and timing ---------------------------------------------------------------------
    @contextmanager
    def capture(self, stream: torch.cuda.Stream):
        """Capture everything this context enqueues on `stream` into a Graph."""
        g = Graph(self)
        _check(self._lib.pk_graph_begin(self.handle, _stream(stream)))
        try:
            yield g
        except BaseException:
            h = ctypes.c_void_p()
            self._lib.pk_graph_end(self.handle, _stream(stream), ctypes.byref(h))
            if h:
                self._lib.pk_graph_destroy(h)
            raise
        h = ctypes.c_void_p()
        _check(self._lib.pk_graph_end(self.handle, _stream(stream), ctypes.byref(h)))
        g.handle = h

    def timer_start(self, stream=None):
        _check(self._lib.pk_timer_start(self.handle, _stream(stream)))

    def timer_stop(self, stream=None) -> float:
        ms = ctypes.c_double()
        _check(self._lib.pk_timer_stop(self.handle, _stream(stream), ctypes.byref(ms)))
        return float(ms.value)

    def cache_flush(self, stream=None):
        _check(self._lib.pk_cache_flush(self.handle, _stream(stream)))

    STREAM_BLOCKS = 2048     # PK_STREAM_BLOCKS

    def stream_probe(self, kind, src, dst, stream=None):
        """pk_stream_probe: kind "read" (dst: STREAM_BLOCKS block sums) or "copy", or either
        with non-temporal accesses ("read_nt", "copy_nt")."""
        _check(self._lib.pk_stream_probe(self.handle, {"read": 0, "copy": 1, "read_nt": 2, "copy_nt": 3}[kind],
                                         _ptr(src), _ptr(dst), src.numel(), _stream(stream)))
        return dst


class Graph:
    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.handle = None

    def launch(self, stream=None):
        _check(self.ctx._lib.pk_graph_launch(self.handle, _stream(stream)))

    def time(self, reps: int, stream=None) -> float:
        ms = ctypes.c_double()
        _check(self.ctx._lib.pk_graph_time(self.ctx.handle, self.handle, int(reps), _stream(stream),
                                           ctypes.byref(ms)))
        return float(ms.value)

    def destroy(self):
        if self.handle:
            self.ctx._lib.pk_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    """The shared Context of a device (created on first use)."""
    if device is None:
        device = torch.cuda.current_device()
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]
