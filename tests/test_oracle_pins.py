"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test ties one oracle function to an independent source: exact rational
brute force (``fractions``), library routines (numpy float64 products,
``numpy.corrcoef``, scipy correlation, torch's bfloat16 cast), closed forms
and invariants of the definitions.  The cases are chosen so that a plausible
slip (a dropped term, a wrong sign or index, a transposed operand, a flipped
stencil, n instead of n-1) fails at least one of them.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage
import scipy.signal
import torch

from oracle import oracle as o
from paper_1810_10496_amd import synth


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


# ----------------------------------------------------------------- GEMM ----

def _frac_gemm(A, B, C, alpha, beta):
    M, K = A.shape
    N = B.shape[1]
    a, b = Fraction(float(alpha)), Fraction(float(beta))
    out = np.empty((M, N), object)
    for i in range(M):
        for j in range(N):
            s = sum(Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(K))
            out[i, j] = a * s + b * Fraction(float(C[i, j]))
    return out


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (2, 3, 1), (3, 2, 17), (5, 4, 3), (7, 6, 9)])
def test_gemm_brute_force_exact_rational(M, N, K):
    rng = np.random.default_rng(M * 100 + N * 10 + K)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    C = rng.standard_normal((M, N)).astype(np.float32)
    alpha, beta = np.float32(1.5), np.float32(-1.2)
    exact = _frac_gemm(A, B, C, alpha, beta)
    r = o.gemm(A, B, C, alpha, beta)
    s = o.gemm_scale(A, B, C, alpha, beta)
    for i in range(M):
        for j in range(N):
            assert abs(r[i, j] - float(exact[i, j])) <= 1e-14 * s[i, j]


@pytest.mark.parametrize("M,N,K", [(17, 63, 65), (129, 127, 3), (64, 64, 64)])
def test_gemm_small_integers_bitexact(M, N, K):
    A = synth.small_ints(11, (M, K))
    B = synth.small_ints(12, (K, N))
    C = synth.small_ints(13, (M, N))
    r = o.gemm(A, B, C, 2.0, 0.5)
    ref = 2 * (A.astype(np.int64) @ B.astype(np.int64)) + C.astype(np.float64) * 0.5
    assert np.array_equal(r, ref)


def test_gemm_matches_numpy_float64():
    A, B, C, alpha, beta = synth.gemm_inputs(96, m=80, k=112)
    r = o.gemm(A, B, C, alpha, beta)
    ref = np.float64(alpha) * (A.astype(np.float64) @ B.astype(np.float64)) \
        + np.float64(beta) * C.astype(np.float64)
    assert rel(r, ref) < 1e-12


def test_gemm_identity_and_permutation():
    A, B, C, alpha, beta = synth.gemm_inputs(33)
    eye = np.eye(33, dtype=np.float32)
    r = o.gemm(eye, B, C, alpha, beta)
    assert np.array_equal(r, np.float64(alpha) * B.astype(np.float64) + np.float64(beta) * C)
    perm = synth.splitmix64(7, 0, 33).argsort()
    P = eye[perm]                      # P @ B = B[perm]
    r = o.gemm(P, B, C, 1.0, 0.0)
    assert np.array_equal(r, B[perm].astype(np.float64))
    r = o.gemm(A, P.T.copy(), C, 1.0, 0.0)  # A @ P^T = columns of A permuted
    assert np.array_equal(r, A[:, perm].astype(np.float64))


def test_gemm_k0_and_beta_only():
    A = np.zeros((4, 1), np.float32)[:, :0]
    B = np.zeros((0, 5), np.float32)
    C = synth.uniform(3, (4, 5))
    r = o.gemm(np.ascontiguousarray(A), B, C, 1.5, 1.2)
    assert np.array_equal(r, np.float64(np.float32(1.2)) * C.astype(np.float64))


# ------------------------------------------------------------ chained ----

def test_gemm3_reduces_to_gemm_with_identity():
    A, B, C, D, alpha, beta = synth.gemm3_inputs(24)
    eye = np.eye(24, dtype=np.float32)
    r = o.gemm3(eye, B, C, D, alpha, beta)        # (I B) C
    assert rel(r, o.gemm(B, C, D, alpha, beta)) < 1e-14
    r = o.gemm3(A, B, eye, D, alpha, beta)        # (A B) I
    assert rel(r, o.gemm(A, B, D, alpha, beta)) < 1e-14


def test_gemm3_matches_numpy_and_associativity():
    A, B, C, D, alpha, beta = synth.gemm3_inputs(40, m=31, k=45, l=29)
    A, B, C = A[:31, :45].copy(), B[:45, :29].copy(), C[:29, :40].copy()
    D = D[:31, :40].copy()
    r = o.gemm3(A, B, C, D, alpha, beta)
    A64, B64, C64 = (x.astype(np.float64) for x in (A, B, C))
    ref1 = np.float64(alpha) * ((A64 @ B64) @ C64) + np.float64(beta) * D
    ref2 = np.float64(alpha) * (A64 @ (B64 @ C64)) + np.float64(beta) * D
    assert rel(r, ref1) < 1e-12 and rel(r, ref2) < 1e-12


def test_gemm3_small_integers_exact():
    A = synth.small_ints(21, (9, 7))
    B = synth.small_ints(22, (7, 5))
    C = synth.small_ints(23, (5, 6))
    D = synth.small_ints(24, (9, 6))
    r = o.gemm3(A, B, C, D, 1.0, 2.0)
    i64 = lambda x: x.astype(np.int64)
    assert np.array_equal(r, (i64(A) @ i64(B) @ i64(C) + 2 * i64(D)).astype(np.float64))


# -------------------------------------------------------------- gemv ----

def test_gemv_rank1_closed_form():
    u = synth.uniform(31, (50,))
    v = synth.uniform(32, (70,))
    A = np.outer(u, v).astype(np.float32)
    x = synth.uniform(33, (70,))
    z = synth.uniform(34, (50,))
    A64 = A.astype(np.float64)
    # y1 = A x and y2 = A^T z computed by the library product
    assert rel(o.gemv(A, x), A64 @ x.astype(np.float64)) < 1e-13
    assert rel(o.gemv_t(A, z), A64.T @ z.astype(np.float64)) < 1e-13
    # rank one: within FP32 rounding of the outer product of u v^T
    y1 = o.gemv(A, x)
    assert rel(y1, u.astype(np.float64) * float(v.astype(np.float64) @ x)) < 1e-6


def test_gemv_bilinear_identity():
    A, x, z = synth.gemv_inputs(300, 257)
    y1 = o.gemv(A, x)
    y2 = o.gemv_t(A, z)
    # z . (A x) == (A^T z) . x
    lhs = float(z.astype(np.float64) @ y1)
    rhs = float(y2 @ x.astype(np.float64))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gemv_identity_permutation_and_ints():
    n = 41
    eye = np.eye(n, dtype=np.float32)
    x = synth.uniform(5, (n,))
    assert np.array_equal(o.gemv(eye, x), x.astype(np.float64))
    perm = synth.splitmix64(9, 0, n).argsort()
    P = eye[perm]
    assert np.array_equal(o.gemv(P, x), x[perm].astype(np.float64))
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n)
    assert np.array_equal(o.gemv_t(P, x), x[inv].astype(np.float64))
    A = synth.small_ints(6, (13, 4097))
    xi = synth.small_ints(7, (4097,))
    zi = synth.small_ints(8, (13,))
    assert np.array_equal(o.gemv(A, xi), (A.astype(np.int64) @ xi.astype(np.int64)).astype(float))
    assert np.array_equal(o.gemv_t(A, zi), (A.T.astype(np.int64) @ zi.astype(np.int64)).astype(float))


# ----------------------------------------------------------- stencils ----

TAPS2 = np.array(synth.CONV2D_TAPS, np.float32)


def test_conv2d_impulse_pins_tap_mapping_and_no_flip():
    H, W, p, q = 9, 11, 4, 5
    g = np.zeros((H, W), np.float32)
    g[p, q] = 1.0
    r = o.conv2d(g, TAPS2)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            # out[i][j] = sum w[di+1][dj+1] in[i+di][j+dj]; the impulse at (p,q)
            # is reached from output (p-di, q-dj) through tap (di, dj)
            assert r[p - di, q - dj] == np.float64(TAPS2[(di + 1) * 3 + (dj + 1)])
    assert np.count_nonzero(r) == 9


def test_conv2d_constant_ramp_and_border():
    H, W = 12, 10
    c = np.float32(3.0)
    r = o.conv2d(np.full((H, W), c, np.float32), TAPS2)
    sw = float(np.sum(TAPS2.astype(np.float64)))
    assert abs(sw - 0.5) < 1e-6          # the coefficients sum to 0.5
    assert np.allclose(r[1:-1, 1:-1], 3.0 * sw, rtol=1e-15, atol=0)
    ramp = np.repeat(np.arange(H, dtype=np.float32)[:, None], W, axis=1)
    r = o.conv2d(ramp, TAPS2)
    w = TAPS2.astype(np.float64).reshape(3, 3)
    row_moment = sum(di * w[di + 1, :].sum() for di in (-1, 0, 1))
    for i in range(1, H - 1):
        assert np.allclose(r[i, 1:-1], i * sw + row_moment, rtol=1e-14, atol=1e-14)
    assert not r[0, :].any() and not r[-1, :].any() and not r[:, 0].any() and not r[:, -1].any()


def test_conv2d_matches_scipy_correlate_and_tiny():
    g, _ = synth.conv2d_inputs(37, 53)
    r = o.conv2d(g, TAPS2)
    ref = scipy.signal.correlate2d(g.astype(np.float64), TAPS2.astype(np.float64).reshape(3, 3),
                                   mode="same")
    assert rel(r[1:-1, 1:-1], ref[1:-1, 1:-1]) < 1e-13
    g3 = synth.uniform(44, (3, 3))
    r3 = o.conv2d(g3, TAPS2)
    assert r3[1, 1] == pytest.approx(float(np.dot(g3.reshape(-1).astype(np.float64),
                                                  TAPS2.astype(np.float64))), rel=1e-15)
    assert np.count_nonzero(r3) == 1


def test_conv2d_dyadic_taps_exact():
    g = synth.small_ints(45, (20, 17), -8, 8)
    w = (synth.small_ints(46, (9,), -8, 8) / 8).astype(np.float32)
    r = o.conv2d(g, w)
    ref = scipy.signal.correlate2d(g.astype(np.float64), w.astype(np.float64).reshape(3, 3),
                                   mode="same")
    assert np.array_equal(r[1:-1, 1:-1], ref[1:-1, 1:-1])


def test_conv3d_matches_scipy_and_faces_zero():
    vol, taps = synth.conv3d_inputs(11, 13, 17)
    r = o.conv3d(vol, taps)
    ref = scipy.ndimage.correlate(vol.astype(np.float64), taps.astype(np.float64).reshape(3, 3, 3),
                                  mode="constant")
    assert rel(r[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1]) < 1e-12
    for face in (r[0], r[-1], r[:, 0], r[:, -1], r[:, :, 0], r[:, :, -1]):
        assert not face.any()


def test_conv3d_middle_plane_taps_reduce_to_2d():
    vol, _ = synth.conv3d_inputs(6, 9, 10)
    taps = np.zeros(27, np.float32)
    taps[9:18] = TAPS2                        # only dz = 0
    r = o.conv3d(vol, taps)
    for z in range(1, 5):
        assert np.array_equal(r[z], o.conv2d(vol[z], TAPS2))


def test_conv3d_impulse():
    vol = np.zeros((5, 6, 7), np.float32)
    vol[2, 3, 3] = 1.0
    taps = synth.uniform(51, (27,), -1, 1)
    r = o.conv3d(vol, taps)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                assert r[2 - dz, 3 - dy, 3 - dx] == np.float64(taps[(dz + 1) * 9 + (dy + 1) * 3 + dx + 1])


# ----------------------------------------------------------- colstats ----

def test_colstats_matches_numpy():
    X, eps = synth.corr_inputs(300, 70)
    mu, sd = o.colstats(X, eps)
    X64 = X.astype(np.float64)
    assert rel(mu, X64.mean(axis=0)) < 1e-13
    assert rel(sd, np.maximum(X64.std(axis=0, ddof=1), 0.1)) < 1e-12


def test_colstats_n2_closed_form_constant_and_floor():
    X = np.array([[1.0, 5.0, 2.0], [4.0, 5.0, 2.05]], np.float32)
    mu, sd = o.colstats(X, 0.1)
    assert mu[0] == 2.5 and sd[0] == pytest.approx(3.0 / np.sqrt(2.0), rel=1e-15)
    assert sd[1] == np.float64(np.float32(0.1))        # constant column: floored
    d = abs(np.float64(X[1, 2]) - np.float64(X[0, 2]))
    assert d / np.sqrt(2) < 0.1 and sd[2] == np.float64(np.float32(0.1))


def test_colstats_shift_invariance():
    X, eps = synth.corr_inputs(200, 16)
    X = (X - X.mean(axis=0)).astype(np.float32)
    shifted = (X.astype(np.float64) + 1e4).astype(np.float32)
    mu0, sd0 = o.colstats(X, eps)
    mu1, sd1 = o.colstats(shifted, eps)
    # exact shift in double of the rounded data, so compare against the data itself
    assert rel(mu1, shifted.astype(np.float64).mean(axis=0)) < 1e-14
    assert rel(sd1, shifted.astype(np.float64).std(axis=0, ddof=1)) < 1e-10
    assert np.allclose(sd0, sd1, rtol=1e-3)    # FP32 rounding of the shifted data only


# --------------------------------------------------------------- corr ----

def test_corr_matches_numpy_corrcoef():
    X, eps = synth.corr_inputs(257, 40)
    R = o.corr(X, eps)
    ref = np.corrcoef(X.astype(np.float64), rowvar=False)
    assert np.max(np.abs(R - ref)) < 1e-13
    assert np.allclose(np.diag(R), 1.0, rtol=0, atol=1e-14)
    assert np.array_equal(R, R.T)


def test_corr_affine_invariance_and_sign():
    X, eps = synth.corr_inputs(128, 12)
    a = np.where(np.arange(12) % 3 == 0, -2.0, 0.5)
    Y = (X.astype(np.float64) * a + 7.0).astype(np.float32)
    R1 = o.corr(Y, eps)
    ref = np.corrcoef(Y.astype(np.float64), rowvar=False)
    assert np.max(np.abs(R1 - ref)) < 1e-13
    R0 = o.corr(X, eps)
    sgn = np.sign(a)[:, None] * np.sign(a)[None, :]
    assert np.max(np.abs(R1 - sgn * R0)) < 1e-5     # FP32 rounding of Y


def test_corr_duplicate_negated_orthogonal_n2():
    n = 16
    Hd = np.array([[1]], np.float64)
    while Hd.shape[0] < n:
        Hd = np.block([[Hd, Hd], [Hd, -Hd]])
    X = np.zeros((n, 5), np.float32)
    X[:, 0] = Hd[:, 1]
    X[:, 1] = Hd[:, 2]          # orthogonal to column 0, both centred
    X[:, 2] = X[:, 0]           # duplicate
    X[:, 3] = -X[:, 0]          # negated
    X[:, 4] = Hd[:, 3] * 3 + 2
    R = o.corr(X, 0.1)
    assert R[0, 1] == 0.0 and R[0, 4] == 0.0 and R[1, 4] == 0.0
    assert R[0, 2] == pytest.approx(1.0, abs=1e-15) and R[0, 3] == pytest.approx(-1.0, abs=1e-15)
    X2 = synth.uniform(61, (2, 6))
    R2 = o.corr(X2, 0.0001)
    assert np.allclose(np.abs(R2), 1.0, atol=1e-12)


def test_corr_row_permutation_and_scale():
    X, eps = synth.corr_inputs(64, 9)
    perm = synth.splitmix64(3, 0, 64).argsort()
    R, S = o.corr(X, eps, with_scale=True)
    Rp = o.corr(X[perm], eps)
    assert np.max(np.abs(R - Rp)) < 1e-14
    assert np.all(S >= np.abs(R) - 1e-15)
    assert np.allclose(np.diag(S), np.diag(R), rtol=1e-15)


def test_corr_constant_column_is_floored_not_forced():
    X, eps = synth.corr_inputs(50, 4)
    X[:, 2] = 3.0
    R = o.corr(X, eps)
    assert np.all(R[2, :] == 0.0) and np.all(R[:, 2] == 0.0)   # centred values are exactly 0


# --------------------------------------------------------------- bf16 ----

def _torch_bf16(x):
    return torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()


def test_bf16_rne_all_rounding_cases_vs_torch():
    # every low-16-bit pattern (all the rounding decisions) under a set of
    # high halves spanning signs, subnormals, normal binades and overflow
    hi = np.array([0x0000, 0x0001, 0x007F, 0x0080, 0x0100, 0x3F80, 0x3F81, 0x4000, 0x4B7F,
                   0x7F00, 0x7F7E, 0x7F7F, 0x8000, 0x8001, 0x807F, 0xBF80, 0xC2FF, 0xFF7F],
                  np.uint32)
    hi = np.concatenate([hi, (synth.splitmix64(77, 0, 64) >> np.uint64(48)).astype(np.uint32)])
    hi = hi[(hi & 0x7F80) != 0x7F80]                      # finite only
    lo = np.arange(1 << 16, dtype=np.uint32)
    bits = (hi[:, None] << 16 | lo[None, :]).reshape(-1)
    x = bits.view(np.float32)
    assert np.array_equal(o.bf16_rne(x).view(np.uint32), _torch_bf16(x).view(np.uint32))


def test_bf16_rne_random_bit_patterns_vs_torch():
    bits = (synth.splitmix64(78, 0, 1 << 21) >> np.uint64(32)).astype(np.uint32)
    bits = bits[(bits & 0x7F800000) != 0x7F800000]
    x = bits.view(np.float32)
    assert np.array_equal(o.bf16_rne(x).view(np.uint32), _torch_bf16(x).view(np.uint32))


def test_split_bf16_reconstruction():
    x = np.concatenate([synth.uniform(79, (4096,)), synth.normal(80, (4096,)) * 1e3])
    x = x.astype(np.float32)
    hi, lo = o.split_bf16(x)
    assert np.array_equal(hi, _torch_bf16(x))
    assert np.array_equal(lo, _torch_bf16((x - hi).astype(np.float32)))
    err = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0 ** -16 * np.abs(x.astype(np.float64)))


def test_gemm_split3_exact_for_bf16_representable_inputs():
    A = synth.small_ints(81, (10, 12))
    B = synth.small_ints(82, (12, 8))
    C = synth.small_ints(83, (10, 8))
    assert np.array_equal(o.gemm_split3(A, B, C, 1.0, 2.0), o.gemm(A, B, C, 1.0, 2.0))
    A, B, C, a, b = synth.gemm_inputs(16)
    d = o.gemm_split3(A, B, C, a, b) - o.gemm(A, B, C, a, b)
    # dropping lo*lo costs at most 2^-16 relative per product
    assert np.max(np.abs(d) / o.gemm_scale(A, B, C, a, b)) < 2.0 ** -15


# ------------------------------------------------------------ metric ----

def test_max_err_metric():
    r = np.array([1.0, -2.0, 0.0])
    s = np.array([1.0, 2.0, 0.0])
    assert o.max_err(np.array([1.0, -2.0, 0.0]), r, s) == 0.0
    assert o.max_err(np.array([1.5, -2.0, 0.0]), r, s) == 0.5
    assert o.max_err(np.array([1.0, -2.0, 1e-30]), r, s) == np.inf


# ------------------------------------------- covariance, rank-k, gesummv, mvt ----

def test_covar_matches_numpy_cov_and_relates_to_corr():
    X, eps = synth.corr_inputs(200, 30)
    C = o.covar(X)
    assert np.max(np.abs(C - np.cov(X.astype(np.float64), rowvar=False))) < 1e-12
    mu, sd = o.colstats(X, eps)
    assert np.allclose(np.diag(C), sd ** 2, rtol=1e-13)        # no floor triggers here
    R = o.corr(X, eps)
    assert np.max(np.abs(C / np.outer(sd, sd) - R)) < 1e-13
    Xs = (X.astype(np.float64) + 3.0).astype(np.float32)
    assert np.max(np.abs(o.covar(Xs) - np.cov(Xs.astype(np.float64), rowvar=False))) < 1e-11


def test_syrk_and_syr2k_match_numpy_and_each_other():
    A = synth.uniform(301, (37, 23))
    B = synth.uniform(302, (37, 23))
    C = synth.uniform(303, (37, 37))
    A64, B64, C64 = (x.astype(np.float64) for x in (A, B, C))
    a, b = np.float32(1.5), np.float32(-0.75)
    r = o.syrk(A, C, a, b)
    assert np.max(np.abs(r - (np.float64(a) * A64 @ A64.T + np.float64(b) * C64))) < 1e-12
    r2 = o.syr2k(A, B, C, a, b)
    assert np.max(np.abs(r2 - (np.float64(a) * (A64 @ B64.T + B64 @ A64.T) + np.float64(b) * C64))) < 1e-12
    # syr2k(A, A) = 2 syrk product; a symmetric C gives a symmetric result
    assert np.max(np.abs(o.syr2k(A, A, C, 1.0, 0.0) - 2 * o.syrk(A, C, 1.0, 0.0))) < 1e-12
    Cs = ((C64 + C64.T) / 2).astype(np.float32)
    rs = o.syrk(A, Cs, a, b)
    assert np.array_equal(rs, rs.T)
    ints = synth.small_ints(304, (9, 11))
    ci = synth.small_ints(305, (9, 9))
    assert np.array_equal(o.syrk(ints, ci, 2.0, 1.0),
                          (2 * ints.astype(np.int64) @ ints.T.astype(np.int64) + ci).astype(np.float64))


def test_gesummv_and_mvt_closed_forms():
    N = 61
    A = synth.uniform(311, (N, N))
    B = synth.uniform(312, (N, N))
    x = synth.uniform(313, (N,))
    A64, B64, x64 = (v.astype(np.float64) for v in (A, B, x))
    y = o.gesummv(A, B, x, 1.5, 1.2)
    assert np.max(np.abs(y - (np.float64(np.float32(1.5)) * A64 @ x64 + np.float64(np.float32(1.2)) * B64 @ x64))) < 1e-12
    assert np.array_equal(o.gesummv(A, A, x, 1.0, -1.0), np.zeros(N))     # (A - A) x exactly
    y1, y2, x1, x2 = (synth.uniform(314 + i, (N,)) for i in range(4))
    o1, o2 = o.mvt(A, y1, y2, x1, x2)
    assert np.max(np.abs(o1 - (x1 + A64 @ y1.astype(np.float64)))) < 1e-12
    assert np.max(np.abs(o2 - (x2 + A64.T @ y2.astype(np.float64)))) < 1e-12
    assert np.allclose(o1 - x1, o.gemv(A, y1), rtol=0, atol=1e-13)


# ------------------------------------------------------------------ FDTD ----

def _fdtd_inputs(NX, NY, T, seed):
    return (synth.uniform(seed, (T,)), synth.uniform(seed + 1, (NX, NY), -1, 1),
            synth.uniform(seed + 2, (NX, NY), -1, 1), synth.uniform(seed + 3, (NX, NY), -1, 1))


def test_fdtd_zero_fields_stay_zero_and_boundary_takes_source():
    NX, NY, T = 9, 7, 5
    z = np.zeros((NX, NY), np.float32)
    ex, ey, hz = o.fdtd2d(np.zeros(T, np.float32), z, z, z)
    assert not ex.any() and not ey.any() and not hz.any()
    fict, ex0, ey0, hz0 = _fdtd_inputs(NX, NY, T, 321)
    ex, ey, hz = o.fdtd2d(fict, ex0, ey0, hz0)
    assert np.array_equal(ey[0], np.full(NY, np.float64(fict[-1])))       # row 0 = source of the last step


def test_fdtd_is_linear():
    fict, ex0, ey0, hz0 = _fdtd_inputs(11, 13, 6, 331)
    a = o.fdtd2d(fict, ex0, ey0, hz0)
    b = o.fdtd2d(*(v * 2 for v in (fict, ex0, ey0, hz0)))
    for p, q in zip(a, b):
        assert np.max(np.abs(q - 2 * p)) < 1e-12


C07 = float(np.float32(0.7))     # the GPU multiplies by the FP32 value of 0.7


def test_fdtd_single_step_light_cone_pins_signs_and_offsets():
    # one hz impulse, everything else zero, one step: the update rules fix where
    # (and with which sign and weight) the impulse appears
    NX, NY, p, q = 7, 8, 3, 4
    z = np.zeros((NX, NY), np.float32)
    hz0 = z.copy()
    hz0[p, q] = 1.0
    ex, ey, hz = o.fdtd2d(np.zeros(1, np.float32), z, z, hz0)
    # ey[i][j] -= 0.5 (hz[i][j] - hz[i-1][j]): touched at (p, q) and (p+1, q)
    want_ey = np.zeros((NX, NY))
    want_ey[p, q], want_ey[p + 1, q] = -0.5, 0.5
    assert np.array_equal(ey, want_ey)
    want_ex = np.zeros((NX, NY))
    want_ex[p, q], want_ex[p, q + 1] = -0.5, 0.5
    assert np.array_equal(ex, want_ex)
    # hz[i][j] -= 0.7 (ex[i][j+1] - ex[i][j] + ey[i+1][j] - ey[i][j]) with the new ex, ey
    want_hz = np.zeros((NX, NY))
    for i in range(NX - 1):
        for j in range(NY - 1):
            want_hz[i, j] = hz0[i, j] - C07 * (want_ex[i, j + 1] - want_ex[i, j] + want_ey[i + 1, j] - want_ey[i, j])
    want_hz[NX - 1, :] = hz0[NX - 1, :]
    want_hz[:, NY - 1] = hz0[:, NY - 1]
    assert np.max(np.abs(hz - want_hz)) < 1e-15
    assert hz[p, q] == pytest.approx(1.0 - 0.7 * 2.0)          # -(-0.5) - (-0.5): both neighbours pull
    assert hz[p, q] == 1.0 - C07 * 2.0                          # with the FP32 coefficient the GPU uses
    assert np.count_nonzero(hz) == 5


def _dependence_support(NX, NY, T, p, q):
    """Cells whose final value can depend on hz[p][q] at the start, by boolean
    propagation of the update rules' read sets (no arithmetic)."""
    dx = np.zeros((NX, NY), bool)
    dy = np.zeros((NX, NY), bool)
    dh = np.zeros((NX, NY), bool)
    dh[p, q] = True
    for _ in range(T):
        dy[0, :] = False                                   # row 0 is overwritten by the source
        dy[1:, :] |= dh[1:, :] | dh[:-1, :]
        dx[:, 1:] |= dh[:, 1:] | dh[:, :-1]
        dh[:-1, :-1] |= dx[:-1, 1:] | dx[:-1, :-1] | dy[1:, :-1] | dy[:-1, :-1]
    return dx, dy, dh


def test_fdtd_scales_follow_the_domain_of_dependence_and_bound():
    """Error scales of the FDTD oracle.  After one step from a single hz impulse (everything
    else zero) an element's scale is the impulse's magnitude 1 wherever an update read it,
    1 + 2c at the impulse (its own update's terms), 0 elsewhere; after several steps the
    scales are non-zero exactly on the impulse's domain of influence, found by propagating
    the update rules' read sets.  On random fields the scale bounds |r| everywhere and the
    error of an FP32 evaluation (plain and with the H update fused) element by element."""
    NX, NY, p, q = 7, 8, 3, 4
    z = np.zeros((NX, NY), np.float32)
    hz0 = z.copy()
    hz0[p, q] = 1.0
    (ex, ey, hz), (sx, sy, sh) = o.fdtd2d(np.zeros(1, np.float32), z, z, hz0, with_scale=True)
    want = np.zeros((NX, NY))
    want[p, q] = want[p + 1, q] = 1.0
    assert np.array_equal(sy, want)
    want = np.zeros((NX, NY))
    want[p, q] = want[p, q + 1] = 1.0
    assert np.array_equal(sx, want)
    want = np.zeros((NX, NY))
    want[p, q] = 1.0 + C07 * 2.0
    want[p - 1, q] = want[p + 1, q] = want[p, q - 1] = want[p, q + 1] = 1.0
    assert np.array_equal(sh, want)
    # several steps on a larger grid: the scales' support is the domain of influence
    NX, NY, p, q, T = 23, 19, 9, 7, 6
    hz0 = np.zeros((NX, NY), np.float32)
    hz0[p, q] = 1.0
    z = np.zeros((NX, NY), np.float32)
    vals, scales = o.fdtd2d(np.zeros(T, np.float32), z, z, hz0, with_scale=True)
    for v, sc, dep in zip(vals, scales, _dependence_support(NX, NY, T, p, q)):
        assert np.array_equal(sc > 0, dep)
        assert not np.any(v[~dep])
    # random fields, several steps: |r| <= s, and an FP32 evaluation stays within a few
    # roundings per step of s
    T = 8
    fict, ex0, ey0, hz0 = _fdtd_inputs(31, 29, T, 341)
    refs, scales = o.fdtd2d(fict, ex0, ey0, hz0, with_scale=True)
    for r, sc in zip(refs, scales):
        assert np.all(np.abs(r) <= sc * (1 + 1e-15))
    half, c = np.float32(0.5), np.float32(0.7)
    for fused in (False, True):
        ex, ey, hz = (v.astype(np.float32).copy() for v in (ex0, ey0, hz0))
        for t in range(T):
            ey[0, :] = fict[t]
            ey[1:, :] -= half * (hz[1:, :] - hz[:-1, :])
            ex[:, 1:] -= half * (hz[:, 1:] - hz[:, :-1])
            s = ex[:-1, 1:] - ex[:-1, :-1] + ey[1:, :-1] - ey[:-1, :-1]
            if fused:   # one rounding of hz - c*s (exact in FP64 for FP32 operands)
                hz[:-1, :-1] = (hz[:-1, :-1].astype(np.float64) - np.float64(c) * s).astype(np.float32)
            else:
                hz[:-1, :-1] -= c * s
        errs = [o.max_err(g, r, sc) for g, r, sc in zip((ex, ey, hz), refs, scales)]
        assert 0 < max(errs) <= 1e-6 * (1 + T), errs


def test_gemm_split3_drops_exactly_the_lo_lo_term():
    """a = b = 1 + 2^-9: hi = 1 (RNE to 8 significant bits), lo = 2^-9, so the three-term
    product is 1 + 2^-8 and the dropped lo*lo is 2^-18 (the full product is 1 + 2^-8 + 2^-18)."""
    a = np.array([[1.0 + 2.0 ** -9]], np.float32)
    hi, lo = o.split_bf16(a)
    assert hi[0, 0] == 1.0 and lo[0, 0] == 2.0 ** -9
    got = o.gemm_split3(a, a, np.zeros((1, 1), np.float32), 1.0, 0.0)
    assert got[0, 0] == 1.0 + 2.0 ** -8
    assert o.gemm(a, a, np.zeros((1, 1), np.float32), 1.0, 0.0)[0, 0] == 1.0 + 2.0 ** -8 + 2.0 ** -18
    # accumulated over K: each product drops its own lo*lo
    K = 6
    A = np.full((1, K), 1.0 + 2.0 ** -9, np.float32)
    B = np.full((K, 1), 1.0 + 2.0 ** -9, np.float32)
    assert o.gemm_split3(A, B, np.zeros((1, 1), np.float32), 1.0, 0.0)[0, 0] == K * (1.0 + 2.0 ** -8)
