"""GPU parity of the one-launch variants (FUSE = 1) of the transposed matvec, the
pair and the column statistics: the last block of each group folds the partials, so
there is no second launch.  Checked against the FP64 oracle on ragged shapes
(groups of one block included), bitwise on small-integer inputs, with workspaces
that hold garbage or a previous call's state, under graph replay (one ticket tag
replayed), for MVT's accumulate form, inside the correlation and covariance, and
with a workspace too little aligned for them (the built-in default runs instead)."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_1810_10496_amd import api, codegen, synth
from paper_1810_10496_amd.tuner import gate

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

VARIANTS = [
    ("gemv_t", dict(ROWS=64, WAVES=4, VEC=4, UNROLL=16, ORDER=0, FUSE=1)),
    ("gemv_t", dict(ROWS=256, WAVES=8, VEC=1, UNROLL=8, ORDER=1, FUSE=1)),
    ("gemv_t", dict(ROWS=16, WAVES=1, VEC=2, UNROLL=4, ORDER=0, FUSE=1)),
    ("gemv_pair", dict(ROWS=64, WAVES=4, VEC=4, UNROLL=16, ORDER=0, FUSE=1)),
    ("gemv_pair", dict(ROWS=256, WAVES=8, VEC=2, UNROLL=32, ORDER=1, FUSE=1)),
    ("gemv_pair", dict(ROWS=16, WAVES=2, VEC=1, UNROLL=8, ORDER=0, FUSE=1)),
    ("colstats", dict(VEC=4, WAVES=4, ROWS=64, ORDER=0, FUSE=1)),
    ("colstats", dict(VEC=1, WAVES=8, ROWS=256, ORDER=1, FUSE=1)),
    ("colstats", dict(VEC=2, WAVES=1, ROWS=16, ORDER=0, FUSE=1)),
]
# (M, N): several row blocks and strips with ragged ends, one row block, one strip, 1 x 1
GEMV_SHAPES = [(77, 130), (1000, 257), (300, 4097), (16, 64), (5000, 33), (1, 1), (2048, 2048)]
COLSTATS_SHAPES = [(130, 70), (1000, 257), (2, 5), (4096, 300), (5000, 64), (16, 1)]


def g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def built():
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(lambda v: codegen.compile_variant(v[0], v[1]), VARIANTS))


@pytest.fixture(scope="module")
def ctx():
    return api.context(0)


class selected:
    """Load a built variant and force it for its family while in the block."""

    def __init__(self, ctx, fam, code):
        self.ctx, self.fam, self.code = ctx, fam, code

    def __enter__(self):
        assert gate.check(self.code) is None
        self.vid = self.ctx.variant_load(self.code)
        f, k, _ = self.ctx.variant_info(self.vid)
        assert f == api.FAMILY_IDS[self.fam] and k[15] == 1       # knob X3: one launch
        self.ctx.variant_select(self.fam, self.vid)
        return self.vid

    def __exit__(self, *exc):
        self.ctx.variant_select(self.fam, -1)
        self.ctx.variant_unload(self.vid)


def run(ctx, fam, M, N, seed=0, ws=None):
    """One call of the family's operation on seeded inputs; (outputs, oracle refs, scales)."""
    if fam == "colstats":
        X, eps = synth.corr_inputs(M, N)
        mu, sd = ctx.colstats(g(X), eps, ws=ws)
        mr, sr = o.colstats(X, eps)
        return (h(mu), h(sd)), (mr, sr), (o.colstats(np.abs(X), eps)[0], None)
    A, x, z = synth.gemv_inputs(M, N)
    if seed:
        A = synth.uniform(900 + seed, (M, N))
    if fam == "gemv_t":
        return (h(ctx.gemv_t(g(A), g(z), ws=ws)),), (o.gemv_t(A, z),), (None,)
    y1, y2 = ctx.gemv_pair(g(A), g(x), g(z), ws=ws)
    return (h(y1), h(y2)), (o.gemv(A, x), o.gemv_t(A, z)), (None, None)


def tol(fam, k):
    return (1e-6, 1e-5)[k] if fam == "colstats" else 1e-4


@pytest.mark.parametrize("i", range(len(VARIANTS)))
def test_one_launch_vs_oracle(ctx, built, i):
    fam, knobs = VARIANTS[i]
    print("[case] one-launch", fam, knobs, flush=True)
    shapes = COLSTATS_SHAPES if fam == "colstats" else GEMV_SHAPES
    with selected(ctx, fam, built[i].code):
        for M, N in shapes:
            outs, refs, scales = run(ctx, fam, M, N)
            for k, (out, ref, sc) in enumerate(zip(outs, refs, scales)):
                assert o.max_err(out, ref, sc) <= tol(fam, k), (M, N, k)
            again, _, _ = run(ctx, fam, M, N)
            for out, out2 in zip(outs, again):
                assert np.array_equal(out, out2), (M, N)           # fixed fold order
        if fam != "colstats":
            # small integers: every partial sum is exact, so the result is the oracle's bit for bit
            for M, N in ((300, 257), (1000, 130)):
                A = synth.small_ints(871, (M, N))
                x = synth.small_ints(872, N)
                z = synth.small_ints(873, M)
                if fam == "gemv_t":
                    assert np.array_equal(h(ctx.gemv_t(g(A), g(z))).astype(np.float64), o.gemv_t(A, z))
                else:
                    y1, y2 = ctx.gemv_pair(g(A), g(x), g(z))
                    assert np.array_equal(h(y1).astype(np.float64), o.gemv(A, x))
                    assert np.array_equal(h(y2).astype(np.float64), o.gemv_t(A, z))


@pytest.mark.parametrize("fam", ["gemv_t", "gemv_pair", "colstats"])
def test_one_launch_workspace_state(ctx, built, fam):
    """Whatever the workspace held before (zeros, all ones bits, a constant float, random
    bytes, a previous call's partials and cleared tickets), the call is right."""
    print("[case] one-launch workspace state", fam, flush=True)
    i = [k for k, v in enumerate(VARIANTS) if v[0] == fam][0]
    M, N = (1000, 257)
    kern = {"gemv_t": "gemv_t", "gemv_pair": "gemv_pair", "colstats": "colstats"}[fam]
    nb = api.Context.workspace_bytes(kern, (M, N))
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    rng = np.random.default_rng(5)
    fills = [lambda: ws.zero_(), lambda: ws.fill_(255), lambda: ws.view(torch.float32)[: nb // 4].fill_(1.0),
             lambda: ws.copy_(g(rng.integers(0, 256, nb, dtype=np.uint8))), lambda: None]
    with selected(ctx, fam, built[i].code):
        ref_outs = None
        for fill in fills:
            fill()
            torch.cuda.synchronize()
            outs, refs, scales = run(ctx, fam, M, N, ws=ws)
            for k, (out, ref, sc) in enumerate(zip(outs, refs, scales)):
                assert o.max_err(out, ref, sc) <= tol(fam, k)
            if ref_outs is None:
                ref_outs = outs
            for out, r in zip(outs, ref_outs):
                assert np.array_equal(out, r)


def test_one_launch_graph_replay(ctx, built):
    """A captured call replays one ticket tag: each replay, with new inputs copied in
    between, matches the oracle for those inputs."""
    print("[case] one-launch graph replay", flush=True)
    codes = {fam: built[[k for k, v in enumerate(VARIANTS) if v[0] == fam][0]].code
             for fam in ("gemv_t", "gemv_pair", "colstats")}
    vids = {}
    for fam, code in codes.items():
        vids[fam] = ctx.variant_load(code)
        ctx.variant_select(fam, vids[fam])
    try:
        M, N = 700, 500
        s = torch.cuda.Stream()
        Ab = torch.empty((M, N), device=DEV)
        xb, zb = torch.empty(N, device=DEV), torch.empty(M, device=DEV)
        Xb = torch.empty((M, N), device=DEV)
        yt, y1, y2 = torch.empty(N, device=DEV), torch.empty(M, device=DEV), torch.empty(N, device=DEV)
        mu, sd = torch.empty(N, device=DEV), torch.empty(N, device=DEV)
        wt = torch.empty(api.Context.workspace_bytes("gemv_t", (M, N)), dtype=torch.uint8, device=DEV)
        wp = torch.empty(api.Context.workspace_bytes("gemv_pair", (M, N)), dtype=torch.uint8, device=DEV)
        wc = torch.empty(api.Context.workspace_bytes("colstats", (M, N)), dtype=torch.uint8, device=DEV)
        torch.cuda.synchronize()
        with ctx.capture(s) as graph:
            ctx.gemv_t(Ab, zb, yt, ws=wt, stream=s)
            ctx.gemv_pair(Ab, xb, zb, y1, y2, ws=wp, stream=s)
            ctx.colstats(Xb, 0.1, mu, sd, ws=wc, stream=s)
        for rep in range(3):
            A = synth.uniform(950 + rep, (M, N))
            x, z = synth.uniform(960 + rep, N), synth.uniform(970 + rep, M)
            X, eps = synth.corr_inputs(M, N, workload=4 + rep)
            Ab.copy_(g(A)); xb.copy_(g(x)); zb.copy_(g(z)); Xb.copy_(g(X))
            torch.cuda.synchronize()
            graph.launch(s)
            s.synchronize()
            assert o.max_err(h(yt), o.gemv_t(A, z)) <= 1e-4, rep
            assert o.max_err(h(y1), o.gemv(A, x)) <= 1e-4 and o.max_err(h(y2), o.gemv_t(A, z)) <= 1e-4, rep
            mr, sr = o.colstats(X, np.float32(0.1))
            assert o.max_err(h(mu), mr, o.colstats(np.abs(X), 0.1)[0]) <= 1e-6 and o.max_err(h(sd), sr) <= 1e-5, rep
        graph.destroy()
    finally:
        for fam, vid in vids.items():
            ctx.variant_select(fam, -1)
            ctx.variant_unload(vid)


@pytest.mark.parametrize("N", [7, 300, 1000, 2048])
def test_one_launch_mvt(ctx, built, N):
    """MVT's accumulate form (x1 += A y1, x2 += A^T y2) on a one-launch pair variant."""
    print("[case] one-launch mvt", N, flush=True)
    for i, (fam, _) in enumerate(VARIANTS):
        if fam != "gemv_pair":
            continue
        with selected(ctx, fam, built[i].code):
            A = synth.uniform(431, (N, N))
            y1, y2, x1, x2 = (synth.uniform(432 + k, (N,)) for k in range(4))
            gx1, gx2 = g(x1), g(x2)
            ctx.mvt(g(A), g(y1), g(y2), gx1, gx2)
            r1, r2 = o.mvt(A, y1, y2, x1, x2)
            s1, s2 = o.mvt(np.abs(A), np.abs(y1), np.abs(y2), np.abs(x1), np.abs(x2))
            assert o.max_err(h(gx1), r1, s1) <= 1e-4 and o.max_err(h(gx2), r2, s2) <= 1e-4


@pytest.mark.parametrize("prec", ["fp32", "bf16", "split"])
def test_one_launch_inside_corr_and_covar(ctx, built, prec):
    print("[case] one-launch colstats in corr/covar", prec, flush=True)
    t = {"fp32": 1e-4, "bf16": 2e-2, "split": 1e-5}[prec]
    for i, (fam, _) in enumerate(VARIANTS):
        if fam != "colstats":
            continue
        with selected(ctx, fam, built[i].code):
            for n, m in ((257, 129), (1000, 300)):
                X, eps = synth.corr_inputs(n, m)
                R, mu, sd = ctx.corr(g(X), eps, prec=prec)
                Rr, S = o.corr(X, eps, with_scale=True)
                Rh = h(R)
                assert o.max_err(Rh, Rr, S) <= t and np.array_equal(Rh, Rh.T)
                C, _ = ctx.covar(g(X), prec=prec)
                Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
                scale = np.abs(Xc).T @ np.abs(Xc) / (n - 1)
                assert o.max_err(h(C), o.covar(X), scale) <= t


def test_one_launch_unaligned_workspace_runs_default(ctx, built):
    """A workspace that is only 4-byte aligned cannot hold the 64-bit tickets: the call
    runs the family's built-in default instead, and is still right."""
    print("[case] one-launch unaligned workspace", flush=True)
    for i, (fam, _) in enumerate(VARIANTS):
        if i % 3:
            continue
        M, N = 300, 257
        nb = api.Context.workspace_bytes(fam if fam != "colstats" else "colstats", (M, N))
        big = torch.empty(nb + 16, dtype=torch.uint8, device=DEV)
        ws = big[4:4 + nb]
        with selected(ctx, fam, built[i].code):
            outs, refs, scales = run(ctx, fam, M, N, ws=ws)
            for k, (out, ref, sc) in enumerate(zip(outs, refs, scales)):
                assert o.max_err(out, ref, sc) <= tol(fam, k)
