"""Python face of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the product path never imports it.  It
shares nothing with the GPU library except the seeded input generators, which
hold no kernel arithmetic.

Every function takes the FP32 numpy arrays the GPU sees and returns float64
results (the exact answer to the GPU's actual problem, up to FP64 rounding).
The operations are the textbook definitions of the paper's kernels
(Sec. 2.2 names them; Sec. 3.4 describes CORR's mean/deviation kernels).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_f32 = ctypes.c_float


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: -O2, OpenMP, no fast-math, no BLAS."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_gemm.argtypes = [_i64, _i64, _i64, _f32, _f32p, _i64, _f32p, _i64, _f32,
                                _f32p, _i64, _f64p]
    lib.oracle_gemm3.argtypes = [_i64, _i64, _i64, _i64, _f32, _f32p, _i64, _f32p, _i64,
                                 _f32p, _i64, _f32, _f32p, _i64, _f64p]
    lib.oracle_gemv.argtypes = [_i64, _i64, _f32p, _i64, _f32p, _f64p]
    lib.oracle_gemv_t.argtypes = [_i64, _i64, _f32p, _i64, _f32p, _f64p]
    lib.oracle_conv2d.argtypes = [_i64, _i64, _f32p, _f32p, _i64, _f64p]
    lib.oracle_conv3d.argtypes = [_i64, _i64, _i64, _f32p, _f32p, _f64p]
    lib.oracle_colstats.argtypes = [_i64, _i64, _f32p, _i64, _f32, _f64p, _f64p]
    lib.oracle_corr.argtypes = [_i64, _i64, _f32p, _i64, _f32, _f64p, ctypes.c_void_p]
    lib.oracle_bf16_rne.argtypes = [_f32]
    lib.oracle_bf16_rne.restype = _f32
    lib.oracle_bf16_rne_array.argtypes = [_i64, _f32p, _f32p]
    lib.oracle_split_bf16.argtypes = [_i64, _f32p, _f32p, _f32p]
    lib.oracle_gemm_split3.argtypes = [_i64, _i64, _i64, _f32, _f32p, _i64, _f32p, _i64,
                                       _f32, _f32p, _i64, _f64p]
    lib.oracle_covar.argtypes = [_i64, _i64, _f32p, _i64, _f64p]
    lib.oracle_syrk.argtypes = [_i64, _i64, _f32, _f32p, _i64, _f32, _f32p, _i64, _f64p]
    lib.oracle_syr2k.argtypes = [_i64, _i64, _f32, _f32p, _i64, _f32p, _i64, _f32, _f32p, _i64, _f64p]
    lib.oracle_gesummv.argtypes = [_i64, _f32, _f32p, _i64, _f32, _f32p, _i64, _f32p, _f64p]
    lib.oracle_mvt.argtypes = [_i64, _f32p, _i64, _f32p, _f32p, _f32p, _f32p, _f64p, _f64p]
    lib.oracle_fdtd2d.argtypes = [_i64, _i64, _i64, _f32p, _f32p, _f32p, _f32p, _f64p, _f64p, _f64p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    _lib = lib
    return lib


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the previous count."""
    lib = _load()
    prev = int(lib.oracle_num_threads())
    lib.oracle_set_threads(int(n))
    return prev


def gemm(A, B, C, alpha, beta):
    """alpha * A @ B + beta * C  (GEMM)."""
    A, B, C = _c32(A), _c32(B), _c32(C)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2 and C.shape == (M, N)
    out = np.empty((M, N), np.float64)
    _load().oracle_gemm(M, N, K, float(np.float32(alpha)), A, K, B, N,
                        float(np.float32(beta)), C, N, out)
    return out


def gemm_scale(A, B, C, alpha, beta):
    """Error scale s: the same product with every term made non-negative."""
    return gemm(np.abs(A), np.abs(B), np.abs(C), abs(float(alpha)), abs(float(beta)))


def gemm3(A, B, Cm, D, alpha, beta):
    """alpha * (A @ B) @ Cm + beta * D with the intermediate kept in FP64."""
    A, B, Cm, D = _c32(A), _c32(B), _c32(Cm), _c32(D)
    M, K = A.shape
    K2, L = B.shape
    L2, N = Cm.shape
    assert K == K2 and L == L2 and D.shape == (M, N)
    out = np.empty((M, N), np.float64)
    _load().oracle_gemm3(M, N, K, L, float(np.float32(alpha)), A, K, B, L, Cm, N,
                         float(np.float32(beta)), D, N, out)
    return out


def gemm3_scale(A, B, Cm, D, alpha, beta):
    return gemm3(np.abs(A), np.abs(B), np.abs(Cm), np.abs(D), abs(float(alpha)),
                 abs(float(beta)))


def gemv(A, x):
    """y1 = A @ x."""
    A, x = _c32(A), _c32(x)
    M, N = A.shape
    assert x.shape == (N,)
    y = np.empty(M, np.float64)
    _load().oracle_gemv(M, N, A, N, x, y)
    return y


def gemv_t(A, z):
    """y2 = A.T @ z."""
    A, z = _c32(A), _c32(z)
    M, N = A.shape
    assert z.shape == (M,)
    y = np.empty(N, np.float64)
    _load().oracle_gemv_t(M, N, A, N, z, y)
    return y


def conv2d(grid, taps):
    """3x3 stencil, no flip, border written as 0."""
    grid, taps = _c32(grid), _c32(taps).reshape(9)
    H, W = grid.shape
    out = np.empty((H, W), np.float64)
    _load().oracle_conv2d(H, W, taps, grid, W, out)
    return out


def conv3d(vol, taps):
    """3x3x3 stencil on a dense D x H x W volume, no flip, faces written as 0."""
    vol, taps = _c32(vol), _c32(taps).reshape(27)
    D, H, W = vol.shape
    out = np.empty((D, H, W), np.float64)
    _load().oracle_conv3d(D, H, W, taps, vol, out)
    return out


def colstats(X, eps):
    """Column mean and (n-1)-normalised deviation floored at eps."""
    X = _c32(X)
    n, m = X.shape
    mean = np.empty(m, np.float64)
    std = np.empty(m, np.float64)
    _load().oracle_colstats(n, m, X, m, float(np.float32(eps)), mean, std)
    return mean, std


def corr(X, eps, with_scale: bool = False):
    """Correlation matrix R (m x m) of the columns of X; optionally its error scale."""
    X = _c32(X)
    n, m = X.shape
    R = np.empty((m, m), np.float64)
    S = np.empty((m, m), np.float64) if with_scale else None
    _load().oracle_corr(n, m, X, m, float(np.float32(eps)), R,
                        S.ctypes.data if with_scale else None)
    return (R, S) if with_scale else R


def bf16_rne(x):
    """Round FP32 values to bfloat16 (returned as FP32 holding the bf16 value)."""
    x = _c32(x)
    out = np.empty_like(x)
    _load().oracle_bf16_rne_array(x.size, x.reshape(-1), out.reshape(-1))
    return out


def split_bf16(x):
    """hi = bf16(x), lo = bf16(x - hi)."""
    x = _c32(x)
    hi = np.empty_like(x)
    lo = np.empty_like(x)
    _load().oracle_split_bf16(x.size, x.reshape(-1), hi.reshape(-1), lo.reshape(-1))
    return hi, lo


def gemm_split3(A, B, C, alpha, beta):
    """Exact value of the three-term split-bf16 product (drops lo*lo)."""
    A, B, C = _c32(A), _c32(B), _c32(C)
    M, K = A.shape
    N = B.shape[1]
    out = np.empty((M, N), np.float64)
    _load().oracle_gemm_split3(M, N, K, float(np.float32(alpha)), A, K, B, N,
                               float(np.float32(beta)), C, N, out)
    return out


def covar(X):
    """Covariance matrix of the columns of X (n-1 normalised)."""
    X = _c32(X)
    n, m = X.shape
    C = np.empty((m, m), np.float64)
    _load().oracle_covar(n, m, X, m, C)
    return C


def syrk(A, C, alpha, beta):
    """alpha * A @ A.T + beta * C (A is N x K)."""
    A, C = _c32(A), _c32(C)
    N, K = A.shape
    out = np.empty((N, N), np.float64)
    _load().oracle_syrk(N, K, float(np.float32(alpha)), A, K, float(np.float32(beta)), C, N, out)
    return out


def syr2k(A, B, C, alpha, beta):
    """alpha * (A @ B.T + B @ A.T) + beta * C."""
    A, B, C = _c32(A), _c32(B), _c32(C)
    N, K = A.shape
    out = np.empty((N, N), np.float64)
    _load().oracle_syr2k(N, K, float(np.float32(alpha)), A, K, B, K, float(np.float32(beta)), C, N, out)
    return out


def gesummv(A, B, x, alpha, beta):
    """alpha * A @ x + beta * B @ x."""
    A, B, x = _c32(A), _c32(B), _c32(x)
    N = A.shape[0]
    y = np.empty(N, np.float64)
    _load().oracle_gesummv(N, float(np.float32(alpha)), A, N, float(np.float32(beta)), B, N, x, y)
    return y


def mvt(A, y1, y2, x1, x2):
    """(x1 + A @ y1, x2 + A.T @ y2)."""
    A, y1, y2, x1, x2 = (_c32(v) for v in (A, y1, y2, x1, x2))
    N = A.shape[0]
    o1 = np.empty(N, np.float64)
    o2 = np.empty(N, np.float64)
    _load().oracle_mvt(N, A, N, y1, y2, x1, x2, o1, o2)
    return o1, o2


def fdtd2d(fict, ex, ey, hz, with_scale: bool = False):
    """T = len(fict) steps of the 2D FDTD update; returns (ex, ey, hz) in FP64.  With
    `with_scale`, also each element's error scale (ex, ey, hz): the largest summed
    term magnitude of any update in the element's domain of dependence (its own
    update's and, through the values that update read, every earlier one's), since a
    rounding error travels on through every update that reads it."""
    fict, ex, ey, hz = (_c32(v) for v in (fict, ex, ey, hz))
    NX, NY = ex.shape
    out = [np.empty((NX, NY), np.float64) for _ in range(6 if with_scale else 3)]
    sc = [o.ctypes.data for o in out[3:]] if with_scale else [None, None, None]
    _load().oracle_fdtd2d(len(fict), NX, NY, fict, ex, ey, hz, *out[:3], *sc)
    return (tuple(out[:3]), tuple(out[3:])) if with_scale else tuple(out)


def max_err(gpu, ref, scale=None):
    """max_i |g_i - r_i| / s_i with s the FP64 absolute-value scale (s = |r| if omitted).

    Elements with s_i == 0 count as 0 when g_i == r_i and as inf otherwise.
    """
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    s = np.abs(r) if scale is None else np.asarray(scale, dtype=np.float64)
    d = np.abs(g - r)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d == 0, 0.0, np.inf))
    return float(e.max()) if e.size else 0.0
