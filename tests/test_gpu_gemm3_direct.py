"""The low-precision chained product with T written straight into the second
product's prepared operand (knob EPI of the prepared bf16 / split GEMM): the first
product's epilogue rounds (or splits) T into bf16 rows instead of storing it in FP32
for a separate preparation pass.  Built with the same knobs, the two paths round the
same FP32 values, so D must agree bit for bit; both are checked against the FP64
oracle on ragged shapes (tile edges in every dimension, L below and above a multiple
of 64, L = 1) and bitwise on small-integer inputs."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_1810_10496_amd import api, codegen, synth
from paper_1810_10496_amd.tuner import gate

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"bf16": 2e-2, "split": 1e-5}

# (family, knobs without EPI): the default tile, a 64-wide one with the fragment double
# buffer, a 128 x 128 one (two stages for split)
KNOBS = [
    ("gemm_bf16_ws", {}),
    ("gemm_bf16_ws", dict(BM=64, BN=64, BK=64, WAVES_M=2, WAVES_N=4, ORDER=0, PIPE=2, DSTAGES=4, SCHED=1)),
    ("gemm_split_ws", {}),
    ("gemm_split_ws", dict(BM=128, BN=128, BK=64, WAVES_M=4, WAVES_N=4, ORDER=1, PIPE=1, DSTAGES=2, SCHED=1)),
]
SHAPES = [(65, 33, 47, 70), (300, 260, 129, 257), (1, 1, 1, 1), (100, 37, 129, 1), (513, 300, 200, 128)]


def g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.fixture(scope="module")
def built():
    jobs = [(f, dict(k, EPI=e)) for f, k in KNOBS for e in (0, 1)]
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(lambda j: codegen.compile_variant(j[0], j[1]), jobs))


@pytest.fixture(scope="module")
def ctx():
    return api.context(0)


def run(ctx, fam, code, A, B, Cm, D, alpha, beta, prec):
    assert gate.check(code) is None
    vid = ctx.variant_load(code)
    ctx.variant_select(fam, vid)
    try:
        Dg = g(D)
        ctx.gemm3(g(A), g(B), g(Cm), Dg, alpha, beta, prec=prec)
        torch.cuda.synchronize()
        return Dg.cpu().numpy()
    finally:
        ctx.variant_select(fam, -1)
        ctx.variant_unload(vid)


@pytest.mark.parametrize("i", range(len(KNOBS)))
def test_direct_t_matches_prepared_t_and_oracle(ctx, built, i):
    fam, knobs = KNOBS[i]
    prec = "bf16" if fam == "gemm_bf16_ws" else "split"
    print("[case] gemm3 direct T", fam, knobs, flush=True)
    plain, direct = built[2 * i].code, built[2 * i + 1].code
    for M, N, K, L in SHAPES:
        A = synth.uniform(881, (M, K))
        B = synth.uniform(882, (K, L))
        Cm = synth.uniform(883, (L, N))
        D = synth.uniform(884, (M, N))
        a, b = np.float32(1.5), np.float32(1.2)
        d0 = run(ctx, fam, plain, A, B, Cm, D, a, b, prec)
        d1 = run(ctx, fam, direct, A, B, Cm, D, a, b, prec)
        assert np.array_equal(d0, d1), (M, N, K, L)
        ref = o.gemm3(A, B, Cm, D, a, b)
        # split drops lo*lo, up to 2^-16 of each term's magnitude: over a contraction of
        # L >= 64 terms that stays under the split bar, but a chain whose second product
        # has a handful of terms (L = 1) can reach the per-term bound itself, on both paths
        tol = TOL[prec] if prec == "bf16" or L >= 64 else 3 * 2.0 ** -16
        assert o.max_err(d1, ref, o.gemm3_scale(A, B, Cm, D, a, b)) <= tol, (M, N, K, L)
    # small integers with |T| <= 256: T is exact in bf16, so D is the oracle's bit for bit
    A = synth.small_ints(885, (70, 40))
    B = synth.small_ints(886, (40, 90))
    Cm = synth.small_ints(887, (90, 33))
    D = synth.small_ints(888, (70, 33))
    d1 = run(ctx, fam, direct, A, B, Cm, D, 2.0, 0.5, prec)
    assert np.array_equal(d1.astype(np.float64), o.gemm3(A, B, Cm, D, 2.0, 0.5))
