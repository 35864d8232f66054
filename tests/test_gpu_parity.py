"""GPU parity: every kernel of the library against the FP64 oracle.

Inputs come from the seeded generators; expected values come only from the
oracle.  Error metric: max_i |g_i - r_i| / s_i, where s_i is the FP64 value of
the same expression with every term made non-negative (equal to the plain
relative error on the non-negative workloads).  Bars: FP32 paths 1e-4, BF16
MFMA 2e-2, split-BF16 1e-5.  Integer, index and bit-level work is compared
exactly.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_1810_10496_amd import api, synth

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 2e-2, "split": 1e-5}
DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return api.context(0)


def g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def padded(x, extra):
    """Copy of a 2-D array inside a wider buffer (row stride = cols + extra)."""
    rows, cols = x.shape
    buf = torch.full((rows, cols + extra), float("nan"), dtype=torch.float32, device=DEV)
    buf[:, :cols] = g(x)
    return buf[:, :cols]


# ---------------------------------------------------------------------- GEMM --

GEMM_SHAPES = [(1, 1, 1), (17, 63, 65), (65, 17, 3), (127, 129, 63), (128, 128, 16),
               (200, 130, 257), (512, 512, 512)]


# bf16 / split run two ways: operands prepared once in a workspace (pk_sgemm_ws,
# the default) and rounded inside the product's main loop (pk_sgemm, ws=False)
PREC_PATHS = [("fp32", None), ("bf16", None), ("bf16", False), ("split", None), ("split", False)]


@pytest.mark.parametrize("prec,ws", PREC_PATHS)
@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
def test_gemm_vs_oracle(ctx, prec, ws, M, N, K):
    say("gemm", prec, "workspace" if ws is None else "in-loop", M, N, K)
    A, B, C, alpha, beta = synth.gemm_inputs(N, m=M, k=K)
    ref = o.gemm(A, B, C, alpha, beta)
    s = o.gemm_scale(A, B, C, alpha, beta)
    Cg = g(C)
    ctx.gemm(g(A), g(B), Cg, alpha, beta, prec=prec, ws=ws)
    err = o.max_err(h(Cg), ref, s)
    say("gemm err", err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec,ws", PREC_PATHS)
def test_gemm_small_integers_bitwise(ctx, prec, ws):
    say("gemm ints", prec, ws)
    A = synth.small_ints(101, (96, 200))
    B = synth.small_ints(102, (200, 72))
    C = synth.small_ints(103, (96, 72))
    Cg = g(C)
    ctx.gemm(g(A), g(B), Cg, 2.0, 0.5, prec=prec, ws=ws)
    assert np.array_equal(h(Cg).astype(np.float64), o.gemm(A, B, C, 2.0, 0.5))


@pytest.mark.parametrize("prec", ["bf16", "split"])
def test_gemm_workspace_path_edges(ctx, prec):
    """K = 0, K not a multiple of 64, beta = 0 with a NaN C, too small and misaligned workspaces."""
    say("gemm ws edges", prec)
    C = synth.uniform(7, (5, 6))
    Cg = g(C)
    ctx.gemm(torch.empty((5, 0), device=DEV), torch.empty((0, 6), device=DEV), Cg, 1.5, 1.2, prec=prec)
    assert np.array_equal(h(Cg), (np.float32(1.2) * C).astype(np.float32))
    A, B, _, _, _ = synth.gemm_inputs(70, m=33, k=65)
    Cn = torch.full((33, 70), float("nan"), device=DEV)
    ctx.gemm(g(A), g(B), Cn, 1.5, 0.0, prec=prec)
    z = np.zeros((33, 70), np.float32)
    assert o.max_err(h(Cn), o.gemm(A, B, z, 1.5, 0.0), o.gemm_scale(A, B, z, 1.5, 0.0)) <= TOL[prec]
    need = api.Context.workspace_bytes("gemm", (33, 70, 65), prec)
    a256 = lambda b: (b + 255) // 256 * 256       # noqa: E731
    assert need == (2 if prec == "split" else 1) * (a256(33 * 128 * 2) + a256(70 * 128 * 2))   # Kp = 128
    with pytest.raises(api.PkError):
        ctx.gemm(g(A), g(B), g(z), 1.0, 0.0, prec=prec, ws=torch.empty(need - 1, dtype=torch.uint8, device=DEV))
    big = torch.empty(need + 512, dtype=torch.uint8, device=DEV)
    with pytest.raises(api.PkError) as e:
        ctx.gemm(g(A), g(B), g(z), 1.0, 0.0, prec=prec, ws=big[16:16 + need])
    assert e.value.status == 3                    # PK_ERR_ALIGNMENT


@pytest.mark.parametrize("prec", ["fp32", "split"])
def test_gemm_identity_and_permutation_bitwise(ctx, prec):
    say("gemm identity/permutation", prec)
    n = 96
    _, B, C, _, _ = synth.gemm_inputs(n)
    eye = np.eye(n, dtype=np.float32)
    Cg = g(C)
    ctx.gemm(g(eye), g(B), Cg, 1.0, 0.0, prec=prec)
    out = h(Cg)
    if prec == "fp32":
        assert np.array_equal(out, B)
    else:   # hi + lo of B: within 2^-16 relative, exactly the split reconstruction
        hi, lo = o.split_bf16(B)
        assert np.array_equal(out, (hi.astype(np.float64) + lo).astype(np.float32))
    perm = synth.splitmix64(5, 0, n).argsort()
    P = eye[perm]
    Cg = g(C)
    ctx.gemm(g(P), g(eye), Cg, 1.0, 0.0, prec=prec)
    assert np.array_equal(h(Cg), P)


def test_gemm_beta_zero_does_not_read_c_and_k0(ctx):
    say("gemm beta=0 / K=0")
    A, B, _, _, _ = synth.gemm_inputs(40, m=33, k=29)
    Cg = torch.full((33, 40), float("nan"), device=DEV)
    ctx.gemm(g(A), g(B), Cg, 1.5, 0.0)
    assert o.max_err(h(Cg), o.gemm(A, B, np.zeros((33, 40), np.float32), 1.5, 0.0)) <= 1e-4
    C = synth.uniform(7, (5, 6))
    Cg = g(C)
    ctx.gemm(torch.empty((5, 0), device=DEV), torch.empty((0, 6), device=DEV), Cg, 1.5, 1.2)
    assert np.array_equal(h(Cg), (np.float32(1.2) * C).astype(np.float32))


def test_gemm_strided_rows(ctx):
    say("gemm padded leading dimensions")
    A, B, C, alpha, beta = synth.gemm_inputs(70, m=50, k=90)
    Ap, Bp, Cp = padded(A, 3), padded(B, 5), padded(C, 1)
    ctx.gemm(Ap, Bp, Cp, alpha, beta)
    err = o.max_err(h(Cp), o.gemm(A, B, C, alpha, beta), o.gemm_scale(A, B, C, alpha, beta))
    assert err <= 1e-4


def test_gemm_rejects_bad_arguments(ctx):
    A = torch.zeros((4, 4), device=DEV)
    with pytest.raises(TypeError):
        ctx.gemm(A.double(), A, A)
    with pytest.raises(ValueError):
        ctx.gemm(A, torch.zeros((5, 4), device=DEV), A)
    lib = ctx._lib
    import ctypes
    # ld smaller than the row length -> PK_ERR_SHAPE, nothing enqueued
    st = lib.pk_sgemm(ctx.handle, 0, 4, 4, 4, 1.0, ctypes.c_void_p(A.data_ptr()), 3,
                      ctypes.c_void_p(A.data_ptr()), 4, 0.0, ctypes.c_void_p(A.data_ptr()), 4, None)
    assert st == 2
    # host pointer -> PK_ERR_INVALID_ARG
    host = np.zeros(16, np.float32)
    st = lib.pk_sgemm(ctx.handle, 0, 4, 4, 4, 1.0, ctypes.c_void_p(host.ctypes.data), 4,
                      ctypes.c_void_p(A.data_ptr()), 4, 0.0, ctypes.c_void_p(A.data_ptr()), 4, None)
    assert st == 1
    # extent beyond the allocation -> PK_ERR_INVALID_ARG
    small = torch.zeros(8, device=DEV)
    st = lib.pk_sgemm(ctx.handle, 0, 1000, 1000, 1000, 1.0, ctypes.c_void_p(small.data_ptr()), 1000,
                      ctypes.c_void_p(A.data_ptr()), 1000, 0.0, ctypes.c_void_p(A.data_ptr()), 1000, None)
    assert st == 1


# --------------------------------------------------------------- chained --

@pytest.mark.parametrize("prec", ["fp32", "bf16", "split"])
@pytest.mark.parametrize("M,N,K,L", [(64, 64, 64, 64), (100, 37, 129, 65), (256, 256, 256, 256)])
def test_gemm3_vs_oracle(ctx, prec, M, N, K, L):
    say("gemm3", prec, M, N, K, L)
    A, B, C, D, alpha, beta = synth.gemm3_inputs(N, m=M, k=K, l=L)
    ref = o.gemm3(A, B, C, D, alpha, beta)
    s = o.gemm3_scale(A, B, C, D, alpha, beta)
    Dg = g(D)
    ctx.gemm3(g(A), g(B), g(C), Dg, alpha, beta, prec=prec)
    err = o.max_err(h(Dg), ref, s)
    say("gemm3 err", err)
    assert err <= TOL[prec]


def test_gemm3_small_integers_bitwise_all_precisions(ctx):
    A = synth.small_ints(111, (40, 48))
    B = synth.small_ints(112, (48, 24))
    C = synth.small_ints(113, (24, 36))
    D = synth.small_ints(114, (40, 36))
    ref = o.gemm3(A, B, C, D, 1.0, 2.0)
    assert np.abs(A.astype(np.int64) @ B.astype(np.int64)).max() <= 256   # T exact in bf16
    for prec in ("fp32", "bf16", "split"):
        say("gemm3 ints", prec)
        Dg = g(D)
        ctx.gemm3(g(A), g(B), g(C), Dg, 1.0, 2.0, prec=prec)
        assert np.array_equal(h(Dg).astype(np.float64), ref)


def test_gemm3_full_size_sampled_rows(ctx):
    """2048^3 chained product at the workload size; the oracle checks 24 sampled rows."""
    n = 2048
    A, B, C, D, alpha, beta = synth.gemm3_inputs(n)
    rows = np.sort(synth.splitmix64(3333, 0, 24) % np.uint64(n)).astype(np.int64)
    rows[0], rows[-1] = 0, n - 1
    ref = o.gemm3(A[rows], B, C, D[rows], alpha, beta)
    s = o.gemm3_scale(A[rows], B, C, D[rows], alpha, beta)
    Ag, Bg, Cg = g(A), g(B), g(C)
    for prec in ("fp32", "bf16", "split"):
        say("gemm3 2048", prec)
        Dg = g(D)
        ctx.gemm3(Ag, Bg, Cg, Dg, alpha, beta, prec=prec)
        err = o.max_err(h(Dg)[rows], ref, s)
        say("gemm3 2048 err", prec, err)
        assert err <= TOL[prec]


# ------------------------------------------------------------------ gemv --

GEMV_SHAPES = [(1, 1), (3, 5), (17, 4097), (300, 257), (1000, 1000), (129, 1025)]


@pytest.mark.parametrize("M,N", GEMV_SHAPES)
def test_gemv_family_vs_oracle(ctx, M, N):
    say("gemv family", M, N)
    A, x, z = synth.gemv_inputs(M, N)
    r1, r2 = o.gemv(A, x), o.gemv_t(A, z)
    Ag, xg, zg = g(A), g(x), g(z)
    y1 = ctx.gemv(Ag, xg)
    y2 = ctx.gemv_t(Ag, zg)
    p1, p2 = ctx.gemv_pair(Ag, xg, zg)
    for name, got, ref in (("gemv", y1, r1), ("gemv_t", y2, r2), ("pair.y1", p1, r1), ("pair.y2", p2, r2)):
        err = o.max_err(h(got), ref)
        say(name, err)
        assert err <= 1e-4, name


def test_gemv_integers_bitwise_and_deterministic(ctx):
    say("gemv ints")
    A = synth.small_ints(121, (333, 515))
    x = synth.small_ints(122, (515,))
    z = synth.small_ints(123, (333,))
    Ag, xg, zg = g(A), g(x), g(z)
    y1, y2 = ctx.gemv_pair(Ag, xg, zg)
    assert np.array_equal(h(y1).astype(np.float64), o.gemv(A, x))
    assert np.array_equal(h(y2).astype(np.float64), o.gemv_t(A, z))
    assert np.array_equal(h(ctx.gemv(Ag, xg)).astype(np.float64), o.gemv(A, x))
    assert np.array_equal(h(ctx.gemv_t(Ag, zg)).astype(np.float64), o.gemv_t(A, z))
    Af, xf, zf = synth.gemv_inputs(700, 900)
    a1, a2 = ctx.gemv_pair(g(Af), g(xf), g(zf))
    b1, b2 = ctx.gemv_pair(g(Af), g(xf), g(zf))
    assert np.array_equal(h(a1), h(b1)) and np.array_equal(h(a2), h(b2))


def test_gemv_full_size_and_bilinear_identity(ctx):
    say("gemv pair 4096")
    A, x, z = synth.gemv_inputs(4096)
    Ag, xg, zg = g(A), g(x), g(z)
    y1, y2 = ctx.gemv_pair(Ag, xg, zg)
    r1, r2 = o.gemv(A, x), o.gemv_t(A, z)
    assert o.max_err(h(y1), r1) <= 1e-4 and o.max_err(h(y2), r2) <= 1e-4
    assert o.max_err(h(ctx.gemv(Ag, xg)), r1) <= 1e-4
    assert o.max_err(h(ctx.gemv_t(Ag, zg)), r2) <= 1e-4
    lhs = float(z.astype(np.float64) @ h(y1).astype(np.float64))
    rhs = float(h(y2).astype(np.float64) @ x.astype(np.float64))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_gemv_strided_and_degenerate(ctx):
    say("gemv strided / empty")
    A, x, z = synth.gemv_inputs(77, 130)
    Ap = padded(A, 6)
    assert o.max_err(h(ctx.gemv(Ap, g(x))), o.gemv(A, x)) <= 1e-4
    y1, y2 = ctx.gemv_pair(Ap, g(x), g(z))
    assert o.max_err(h(y2), o.gemv_t(A, z)) <= 1e-4 and o.max_err(h(y1), o.gemv(A, x)) <= 1e-4
    empty = torch.empty((0, 9), device=DEV)
    y = ctx.gemv_t(empty, torch.empty(0, device=DEV))
    assert np.array_equal(h(y), np.zeros(9, np.float32))


# -------------------------------------------------------------- stencils --

TAPS2 = np.array(synth.CONV2D_TAPS, np.float32)


@pytest.mark.parametrize("H,W", [(1, 1), (2, 2), (3, 3), (4, 5), (67, 131), (257, 1030), (1024, 1024)])
def test_conv2d_vs_oracle(ctx, H, W):
    say("conv2d", H, W)
    grid, taps = synth.conv2d_inputs(H, W)
    ref = o.conv2d(grid, taps)
    s = o.conv2d(np.abs(grid), np.abs(taps))
    out = ctx.conv2d(g(grid), taps, out=torch.full((H, W), float("nan"), device=DEV))
    res = h(out)
    assert o.max_err(res, ref, s) <= 1e-4
    assert not res[0].any() and not res[-1].any() and not res[:, 0].any() and not res[:, -1].any()


def test_conv2d_impulse_dyadic_bitwise_and_strided(ctx):
    say("conv2d impulse")
    grid = np.zeros((40, 70), np.float32)
    grid[20, 33] = 1.0
    out = h(ctx.conv2d(g(grid), TAPS2))
    assert np.array_equal(out.astype(np.float64), o.conv2d(grid, TAPS2))
    gi = synth.small_ints(131, (90, 150), -8, 8)
    w = (synth.small_ints(132, (9,), -8, 8) / 8).astype(np.float32)
    assert np.array_equal(h(ctx.conv2d(g(gi), w)).astype(np.float64), o.conv2d(gi, w))
    grid, _ = synth.conv2d_inputs(50, 61)
    inp, outp = padded(grid, 3), padded(np.zeros((50, 61), np.float32), 7)
    ctx.conv2d(inp, TAPS2, out=outp)
    assert o.max_err(h(outp), o.conv2d(grid, TAPS2), o.conv2d(np.abs(grid), np.abs(TAPS2))) <= 1e-4


def test_conv2d_full_size(ctx):
    say("conv2d 4096")
    grid, taps = synth.conv2d_inputs(4096)
    out = h(ctx.conv2d(g(grid), taps))
    assert o.max_err(out, o.conv2d(grid, taps), o.conv2d(np.abs(grid), np.abs(taps))) <= 1e-4


@pytest.mark.parametrize("D,H,W", [(1, 1, 1), (3, 3, 3), (5, 6, 7), (17, 33, 65), (64, 64, 64)])
def test_conv3d_vs_oracle(ctx, D, H, W):
    say("conv3d", D, H, W)
    vol, taps = synth.conv3d_inputs(D, H, W)
    ref = o.conv3d(vol, taps)
    s = o.conv3d(np.abs(vol), np.abs(taps))
    out = ctx.conv3d(g(vol), taps, out=torch.full((D, H, W), float("nan"), device=DEV))
    assert o.max_err(h(out), ref, s) <= 1e-4


def test_conv3d_full_size_and_middle_plane(ctx):
    say("conv3d 256")
    vol, taps = synth.conv3d_inputs(256)
    out = h(ctx.conv3d(g(vol), taps))
    assert o.max_err(out, o.conv3d(vol, taps), o.conv3d(np.abs(vol), np.abs(taps))) <= 1e-4
    t = np.zeros(27, np.float32)
    t[9:18] = TAPS2
    small, _ = synth.conv3d_inputs(6, 20, 33)
    out = h(ctx.conv3d(g(small), t))
    for z in range(1, 5):
        assert o.max_err(out[z], o.conv2d(small[z], TAPS2), o.conv2d(np.abs(small[z]), np.abs(TAPS2))) <= 1e-6


# -------------------------------------------------------------- colstats --

@pytest.mark.parametrize("n,m", [(2, 1), (2, 5), (3, 300), (130, 70), (1000, 257), (2048, 2048)])
def test_colstats_vs_oracle(ctx, n, m):
    say("colstats", n, m)
    X, eps = synth.corr_inputs(n, m)
    mu_r, sd_r = o.colstats(X, eps)
    mu, sd = ctx.colstats(g(X), eps)
    em = o.max_err(h(mu), mu_r, o.colstats(np.abs(X), eps)[0])
    es = o.max_err(h(sd), sd_r)
    say("colstats errs", em, es)
    assert em <= 1e-6 and es <= 1e-5


def test_colstats_shift_constant_column_and_floor(ctx):
    say("colstats shift / constant")
    X, eps = synth.corr_inputs(512, 40)
    X = (X - X.mean(axis=0) + 1e4).astype(np.float32)
    X[:, 3] = 7.25
    mu_r, sd_r = o.colstats(X, eps)
    mu, sd = ctx.colstats(g(X), eps)
    assert o.max_err(h(mu), mu_r) <= 1e-6
    assert o.max_err(h(sd), sd_r) <= 1e-4        # large offset: deviations of ~1 on 1e4
    assert h(sd)[3] == np.float32(eps)


# ------------------------------------------------------------------ corr --

@pytest.mark.parametrize("prec", ["fp32", "bf16", "split"])
@pytest.mark.parametrize("n,m", [(2, 3), (130, 70), (257, 129), (512, 512)])
def test_corr_vs_oracle(ctx, prec, n, m):
    say("corr", prec, n, m)
    X, eps = synth.corr_inputs(n, m)
    Rr, S = o.corr(X, eps, with_scale=True)
    R, mu, sd = ctx.corr(g(X), eps, prec=prec)
    Rh = h(R)
    err = o.max_err(Rh, Rr, S)
    say("corr err", err)
    assert err <= TOL[prec]
    assert np.array_equal(Rh, Rh.T)                       # bitwise symmetric
    assert np.max(np.abs(np.diag(Rh) - 1.0)) <= max(TOL[prec], 1e-5) * 2


def test_corr_full_size_all_precisions(ctx):
    n = m = 2048
    X, eps = synth.corr_inputs(n, m)
    Rr, S = o.corr(X, eps, with_scale=True)
    Xg = g(X)
    for prec in ("fp32", "split", "bf16"):
        say("corr 2048", prec)
        R, _, _ = ctx.corr(Xg, eps, prec=prec)
        Rh = h(R)
        err = o.max_err(Rh, Rr, S)
        say("corr 2048 err", prec, err)
        assert err <= TOL[prec]
        assert np.array_equal(Rh, Rh.T)
        assert np.max(np.abs(np.diag(Rh) - 1.0)) <= 2 * TOL[prec]
        assert np.max(np.abs(Rh)) <= 1.0 + 2 * TOL[prec]


def test_corr_special_columns(ctx):
    say("corr duplicate / negated / constant")
    X, eps = synth.corr_inputs(300, 20)
    X[:, 5] = X[:, 2]
    X[:, 6] = -X[:, 2]
    X[:, 7] = 4.0
    R, _, sd = ctx.corr(g(X), eps, prec="fp32")
    Rh = h(R)
    assert abs(Rh[5, 2] - 1) <= 1e-5 and abs(Rh[6, 2] + 1) <= 1e-5
    assert np.all(Rh[7, :] == 0) and h(sd)[7] == np.float32(eps)


# --------------------------------------------------------------- convert --

def test_convert_bf16_bitwise(ctx):
    say("convert bf16")
    hi16 = np.array([0x0000, 0x0001, 0x0080, 0x3F80, 0x4B7F, 0x7F7F, 0x8000, 0x807F, 0xBF80, 0xC2FF],
                    np.uint32)
    bits = (hi16[:, None] << 16 | np.arange(1 << 16, dtype=np.uint32)[None, :]).reshape(-1)
    x = bits.view(np.float32)
    hi, lo = ctx.convert_bf16(g(x), split=True)
    eh, el = o.split_bf16(x)
    got_hi = (h(hi).astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    got_lo = (h(lo).astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(got_hi.view(np.uint32), eh.view(np.uint32))
    assert np.array_equal(got_lo.view(np.uint32), el.view(np.uint32))


# ------------------------------------------------------------- graphs --

def test_graph_replay_matches_eager(ctx):
    say("graph replay")
    A, B, C, alpha, beta = synth.gemm_inputs(300)
    Av, x, z = synth.gemv_inputs(500, 700)
    grid, taps = synth.conv2d_inputs(200, 300)
    Ag, Bg, Avg, xg, zg, gg = g(A), g(B), g(Av), g(x), g(z), g(grid)
    C0 = g(C)
    s = torch.cuda.Stream()
    Cg = torch.empty_like(C0)
    y1 = torch.empty(500, device=DEV)
    y2 = torch.empty(700, device=DEV)
    out = torch.empty_like(gg)
    ws = torch.empty(api.Context.workspace_bytes("gemv_pair", (500, 700)), dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        Cg.copy_(C0)
    s.synchronize()
    with ctx.capture(s) as graph:
        ctx.gemm(Ag, Bg, Cg, alpha, beta, stream=s)
        ctx.gemv_pair(Avg, xg, zg, y1, y2, ws=ws, stream=s)
        ctx.conv2d(gg, taps, out=out, stream=s)
    eC = ctx.gemm(Ag, Bg, C0.clone(), alpha, beta)
    e1, e2 = ctx.gemv_pair(Avg, xg, zg)
    eo = ctx.conv2d(gg, taps)
    torch.cuda.synchronize()
    eC, e1, e2, eo = h(eC), h(e1), h(e2), h(eo)
    # the eager results (which every replay must reproduce bit for bit) against the oracle
    assert o.max_err(eC, o.gemm(A, B, C, alpha, beta), o.gemm_scale(A, B, C, alpha, beta)) <= 1e-4
    assert o.max_err(e1, o.gemv(Av, x)) <= 1e-4 and o.max_err(e2, o.gemv_t(Av, z)) <= 1e-4
    assert o.max_err(eo, o.conv2d(grid, taps), o.conv2d(np.abs(grid), np.abs(taps))) <= 1e-4
    for rep in range(4):
        with torch.cuda.stream(s):
            Cg.copy_(C0)
        s.synchronize()
        graph.launch(s)
        s.synchronize()
        y1.add_(0.0)   # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(h(Cg), eC), rep
        assert np.array_equal(h(y1), e1) and np.array_equal(h(y2), e2), rep
        assert np.array_equal(h(out), eo), rep
    graph.destroy()


# ---------------------------------------------------------- bandwidth probes --

@pytest.mark.parametrize("n", [0, 3, 4, 1001, 1 << 20, (1 << 20) + 7])
def test_stream_probes(ctx, n):
    """The read probe sums every element exactly once (block sums add up to the total);
    the copy probe copies bitwise, including a ragged tail."""
    say("stream probes", n)
    x = synth.uniform(77, (max(n, 1),))[:n]
    xs = g(x) if n else torch.empty(0, device=DEV)
    for nt in ("", "_nt"):
        sums = torch.full((api.Context.STREAM_BLOCKS,), float("nan"), device=DEV)
        ctx.stream_probe("read" + nt, xs, sums)
        total = float(np.sum(h(sums).astype(np.float64)))
        assert abs(total - float(np.sum(x.astype(np.float64)))) <= 1e-5 * max(1.0, float(np.sum(x)))
        out = torch.full((max(n, 1),), float("nan"), device=DEV)[:n]
        ctx.stream_probe("copy" + nt, xs, out)
        assert np.array_equal(h(out).view(np.uint32), x.view(np.uint32))
