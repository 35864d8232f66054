"""GPU parity of COVAR, SYRK, SYR2K, GESUMMV, MVT (accumulate form) and FDTD-2D
against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_1810_10496_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp32": 1e-4, "bf16": 2e-2, "split": 1e-5}


def g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    return api.context(0)


@pytest.mark.parametrize("prec", ["fp32", "split", "bf16"])
@pytest.mark.parametrize("n,m", [(2, 3), (130, 70), (300, 257), (1024, 512)])
def test_covar_vs_oracle(ctx, prec, n, m):
    print("[case] covar", prec, n, m, flush=True)
    X, _ = synth.corr_inputs(n, m)
    C, mu = ctx.covar(g(X), prec=prec)
    ref = o.covar(X)
    Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
    scale = np.abs(Xc).T @ np.abs(Xc) / max(n - 1, 1)          # sum |d_j d_k| / (n-1)
    Ch = h(C)
    assert o.max_err(Ch, ref, scale) <= TOL[prec]
    assert np.array_equal(Ch, Ch.T)
    assert o.max_err(h(mu), o.colstats(X, 0.1)[0], o.colstats(np.abs(X), 0.1)[0]) <= 1e-6


@pytest.mark.parametrize("N,K", [(1, 1), (33, 17), (130, 257), (1000, 64)])
def test_syrk_syr2k_vs_oracle(ctx, N, K):
    print("[case] syrk/syr2k", N, K, flush=True)
    A = synth.uniform(401, (N, K), -1, 1)
    B = synth.uniform(402, (N, K), -1, 1)
    C = synth.uniform(403, (N, N), -1, 1)          # not symmetric
    a, b = np.float32(1.5), np.float32(-0.75)
    s1 = o.syrk(np.abs(A), np.abs(C), abs(a), abs(b))
    Cg = g(C)
    ctx.syrk(g(A), Cg, a, b)
    assert o.max_err(h(Cg), o.syrk(A, C, a, b), s1) <= 1e-4
    s2 = o.syr2k(np.abs(A), np.abs(B), np.abs(C), abs(a), abs(b))
    Cg = g(C)
    ctx.syr2k(g(A), g(B), Cg, a, b)
    assert o.max_err(h(Cg), o.syr2k(A, B, C, a, b), s2) <= 1e-4
    # beta = 0 does not read C
    Cn = torch.full((N, N), float("nan"), device=DEV)
    ctx.syrk(g(A), Cn, 1.0, 0.0)
    r = h(Cn)
    assert o.max_err(r, o.syrk(A, np.zeros((N, N), np.float32), 1.0, 0.0),
                     o.syrk(np.abs(A), np.zeros((N, N), np.float32), 1.0, 0.0)) <= 1e-4
    assert np.array_equal(r, r.T)


def test_syrk_integers_bitwise(ctx):
    A = synth.small_ints(411, (70, 90))
    C = synth.small_ints(412, (70, 70))
    Cg = g(C)
    ctx.syrk(g(A), Cg, 2.0, 1.0)
    assert np.array_equal(h(Cg).astype(np.float64), o.syrk(A, C, 2.0, 1.0))


@pytest.mark.parametrize("N", [1, 5, 257, 1000, 4096])
def test_gesummv_vs_oracle(ctx, N):
    print("[case] gesummv", N, flush=True)
    A = synth.uniform(421, (N, N))
    B = synth.uniform(422, (N, N))
    x = synth.uniform(423, (N,))
    y = ctx.gesummv(g(A), g(B), g(x), 1.5, 1.2)
    scale = o.gesummv(np.abs(A), np.abs(B), np.abs(x), 1.5, 1.2)
    assert o.max_err(h(y), o.gesummv(A, B, x, 1.5, 1.2), scale) <= 1e-4


@pytest.mark.parametrize("N", [1, 7, 300, 1000, 4096])
def test_mvt_accumulate_vs_oracle(ctx, N):
    print("[case] mvt", N, flush=True)
    A = synth.uniform(431, (N, N))
    y1, y2, x1, x2 = (synth.uniform(432 + i, (N,)) for i in range(4))
    gx1, gx2 = g(x1), g(x2)
    ctx.mvt(g(A), g(y1), g(y2), gx1, gx2)
    r1, r2 = o.mvt(A, y1, y2, x1, x2)
    s1, s2 = o.mvt(np.abs(A), np.abs(y1), np.abs(y2), np.abs(x1), np.abs(x2))
    assert o.max_err(h(gx1), r1, s1) <= 1e-4 and o.max_err(h(gx2), r2, s2) <= 1e-4


@pytest.mark.parametrize("NX,NY,T", [(1, 1, 1), (7, 8, 1), (33, 65, 10), (500, 300, 20), (1000, 1000, 50)])
def test_fdtd2d_vs_oracle(ctx, NX, NY, T):
    print("[case] fdtd2d", NX, NY, T, flush=True)
    fict = synth.uniform(441, (T,))
    ex0 = synth.uniform(442, (NX, NY), -1, 1)
    ey0 = synth.uniform(443, (NX, NY), -1, 1)
    hz0 = synth.uniform(444, (NX, NY), -1, 1)
    ex, ey, hz = ctx.fdtd2d(g(fict), g(ex0), g(ey0), g(hz0))
    refs, scales = o.fdtd2d(fict, ex0, ey0, hz0, with_scale=True)
    # per element, against the largest summed term magnitude in its domain of dependence
    # (errors travel through later updates); FP32 rounding grows with the steps (a step
    # rounds at ~6e-8 of those magnitudes)
    tol = 1e-6 * (1 + T)
    for got, ref, sc in zip((ex, ey, hz), refs, scales):
        assert o.max_err(h(got), ref, sc) <= tol


def test_fdtd2d_in_a_graph_replays(ctx):
    """The time loop captured once and replayed equals the eager loop."""
    NX, NY, T = 200, 300, 8
    fict = g(synth.uniform(451, (T,)))
    base = [g(synth.uniform(452 + i, (NX, NY), -1, 1)) for i in range(3)]
    eager = [t.clone() for t in base]
    ctx.fdtd2d(fict, *eager)
    s = torch.cuda.Stream()
    fields = [t.clone() for t in base]
    torch.cuda.synchronize()
    with ctx.capture(s) as graph:
        ctx.fdtd2d(fict, *fields, stream=s)
    for rep in range(3):
        with torch.cuda.stream(s):
            for f, b in zip(fields, base):
                f.copy_(b)
        s.synchronize()
        graph.launch(s)
        s.synchronize()
        for f, e in zip(fields, eager):
            assert np.array_equal(h(f), h(e)), rep
    graph.destroy()
