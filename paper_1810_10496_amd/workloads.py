"""The measured workloads: problem instances, their inputs and algorithmic cost.

An *instance* is one call of one operation at one size on seeded synthetic
inputs.  The mixed-size batch holds every FP32 operation of the library at
N in {256, 512, 1000, 2048, 4096} (1000 exercises ragged tiles) plus the 3D
stencil on a 256^3 volume; the same instances are what the tuner times.

Algorithmic cost (what rooflines are computed from):
  gemm      2MNK + 3MN flop;  bytes 4(MK + KN + 2MN)
  gemm3     2MKL + 2MLN + 3MN flop (two launches: T = AB, then D)
  gemv/gemv_t   2MN flop;  bytes 4(MN + M + N)
  gemv_pair     4MN flop;  bytes 4(MN + 2M + 2N)
  conv2d    17 (H-2)(W-2) flop;  bytes 8HW (read once, write once)
  conv3d    53 (D-2)(H-2)(W-2) flop;  bytes 8DHW
  colstats  4nm flop;  bytes 4(nm + 2m)
  corr      colstats + m(m+1)/2 * 2n flop (lower triangle only); bytes 4(nm + m^2 + 2m)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import synth

SIZES = (256, 512, 1000, 2048, 4096)
CONV3D_SIZE = 256
WORKLOAD = 5   # seed block of the mixed-size batch


@dataclass
class Instance:
    name: str          # e.g. "gemm/2048"
    op: str            # operation
    families: tuple    # kernel families it launches (tuned per family)
    size: int          # problem size N (largest dimension)
    flops: float
    bytes: float
    bound: str         # "hbm" or "mfma"
    make: callable = None         # (device, copies) -> state
    run: callable = None          # (ctx, state, copy_index, stream) -> None
    footprint: int = 0            # bytes of one copy of the operands
    gemm_flops: float = 0.0       # flops executed by the pk_gemm kernel
    state: dict = field(default_factory=dict)


def _g(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _copies(t, n):
    return [t] + [t.clone() for _ in range(n - 1)]


PREC_FAMILY = {"fp32": "gemm_f32", "bf16": "gemm_bf16_ws", "split": "gemm_split_ws"}


def _gemm(n, prec="fp32", prepared=True):
    """GEMM at n^3.  bf16 / split: `prepared` uses the operands-prepared-once path
    (pk_sgemm_ws, families gemm_*_ws), else the in-loop rounding kernel (pk_sgemm)."""
    def make(dev, copies):
        A, B, C, a, b = synth.gemm_inputs(n, workload=WORKLOAD)
        Ag, Bg = _g(A, dev), _g(B, dev)
        st = dict(A=_copies(Ag, copies), B=_copies(Bg, copies), C=_copies(_g(C, dev), copies),
                  alpha=float(a), beta=float(b), ws=False)
        if prec != "fp32" and prepared:
            st["ws"] = torch.empty(ctx_ws("gemm", (n, n, n), prec), dtype=torch.uint8, device=dev)
        return st

    def run(ctx, s, i, stream):
        ctx.gemm(s["A"][i], s["B"][i], s["C"][i], s["alpha"], s["beta"], prec=prec, ws=s["ws"], stream=stream)

    fl = 2.0 * n ** 3 + 3.0 * n * n
    if prec == "fp32":
        fam, name = "gemm_f32", "gemm"
    elif prepared:
        fam, name = f"gemm_{prec}_ws", f"gemm_{prec}ws"
    else:
        fam, name = f"gemm_{prec}", f"gemm_{prec}"
    return Instance(f"{name}/{n}", name, (fam,), n, fl, 4.0 * 4 * n * n, "mfma", make, run,
                    16 * n * n, gemm_flops=fl)


def _gemm3(n, prec="fp32"):
    def make(dev, copies):
        A, B, C, D, a, b = synth.gemm3_inputs(n, workload=WORKLOAD)
        ws = torch.empty(ctx_ws("gemm3", (n, n, n, n), prec), dtype=torch.uint8, device=dev)
        return dict(A=_copies(_g(A, dev), copies), B=_copies(_g(B, dev), copies),
                    C=_copies(_g(C, dev), copies), D=_copies(_g(D, dev), copies), ws=ws,
                    alpha=float(a), beta=float(b))

    def run(ctx, s, i, stream):
        ctx.gemm3(s["A"][i], s["B"][i], s["C"][i], s["D"][i], s["alpha"], s["beta"], prec=prec, ws=s["ws"],
                  stream=stream)

    fl = 4.0 * n ** 3 + 3.0 * n * n
    name = "gemm3" if prec == "fp32" else f"gemm3_{prec}"
    return Instance(f"{name}/{n}", name, (PREC_FAMILY[prec],), n, fl, 4.0 * 6 * n * n, "mfma", make, run,
                    20 * n * n, gemm_flops=fl)


def _gemv_family(op, n):
    fam = {"gemv": "gemv", "gemv_t": "gemv_t", "gemv_pair": "gemv_pair"}[op]

    def make(dev, copies):
        A, x, z = synth.gemv_inputs(n, workload=WORKLOAD)
        st = dict(A=_copies(_g(A, dev), copies), x=_g(x, dev), z=_g(z, dev),
                  y1=torch.empty(n, device=dev), y2=torch.empty(n, device=dev))
        if op != "gemv":
            st["ws"] = torch.empty(ctx_ws(op, (n, n)), dtype=torch.uint8, device=dev)
        return st

    def run(ctx, s, i, stream):
        if op == "gemv":
            ctx.gemv(s["A"][i], s["x"], s["y1"], stream=stream)
        elif op == "gemv_t":
            ctx.gemv_t(s["A"][i], s["z"], s["y2"], ws=s["ws"], stream=stream)
        else:
            ctx.gemv_pair(s["A"][i], s["x"], s["z"], s["y1"], s["y2"], ws=s["ws"], stream=stream)

    pair = op == "gemv_pair"
    fl = (4.0 if pair else 2.0) * n * n
    by = 4.0 * (n * n + (4 if pair else 2) * n)
    return Instance(f"{op}/{n}", op, (fam,), n, fl, by, "hbm", make, run, 4 * n * n)


def _conv2d(n):
    def make(dev, copies):
        grid, taps = synth.conv2d_inputs(n, workload=WORKLOAD)
        gg = _g(grid, dev)
        return dict(inp=_copies(gg, copies), out=[torch.empty_like(gg) for _ in range(copies)], taps=taps)

    def run(ctx, s, i, stream):
        ctx.conv2d(s["inp"][i], s["taps"], out=s["out"][i], stream=stream)

    return Instance(f"conv2d/{n}", "conv2d", ("conv2d",), n, 17.0 * (n - 2) ** 2, 8.0 * n * n, "hbm",
                    make, run, 8 * n * n)


def _conv3d(n):
    def make(dev, copies):
        vol, taps = synth.conv3d_inputs(n, workload=WORKLOAD)
        vg = _g(vol, dev)
        return dict(inp=_copies(vg, copies), out=[torch.empty_like(vg) for _ in range(copies)], taps=taps)

    def run(ctx, s, i, stream):
        ctx.conv3d(s["inp"][i], s["taps"], out=s["out"][i], stream=stream)

    return Instance(f"conv3d/{n}", "conv3d", ("conv3d",), n, 53.0 * (n - 2) ** 3, 8.0 * n ** 3, "hbm",
                    make, run, 8 * n ** 3)


def _colstats(n):
    def make(dev, copies):
        X, eps = synth.corr_inputs(n, workload=WORKLOAD)
        return dict(X=_copies(_g(X, dev), copies), eps=float(eps), mu=torch.empty(n, device=dev),
                    sd=torch.empty(n, device=dev),
                    ws=torch.empty(ctx_ws("colstats", (n, n)), dtype=torch.uint8, device=dev))

    def run(ctx, s, i, stream):
        ctx.colstats(s["X"][i], s["eps"], s["mu"], s["sd"], ws=s["ws"], stream=stream)

    return Instance(f"colstats/{n}", "colstats", ("colstats",), n, 4.0 * n * n, 4.0 * (n * n + 2 * n),
                    "hbm", make, run, 4 * n * n)


def _corr(n, prec="fp32"):
    def make(dev, copies):
        X, eps = synth.corr_inputs(n, workload=WORKLOAD)
        return dict(X=_copies(_g(X, dev), copies), eps=float(eps), mu=torch.empty(n, device=dev),
                    sd=torch.empty(n, device=dev), R=torch.empty((n, n), device=dev),
                    ws=torch.empty(ctx_ws("corr", (n, n), prec), dtype=torch.uint8, device=dev))

    def run(ctx, s, i, stream):
        ctx.corr(s["X"][i], s["eps"], prec=prec, R=s["R"], mean=s["mu"], std=s["sd"], ws=s["ws"],
                 stream=stream)

    fl = 4.0 * n * n + n * (n + 1) / 2 * 2.0 * n
    name = "corr" if prec == "fp32" else f"corr_{prec}"
    syrk = {"fp32": "syrk_f32", "bf16": "syrk_bf16", "split": "syrk_split"}[prec]
    return Instance(f"{name}/{n}", name, ("colstats", syrk), n, fl, 4.0 * (2 * n * n + 2 * n),
                    "mfma", make, run, 8 * n * n)


def ctx_ws(kernel, dims, prec="fp32"):
    from .api import Context
    return max(Context.workspace_bytes(kernel, dims, prec), 4)


def batch_instances(sizes=SIZES, conv3d_size=CONV3D_SIZE):
    """Every instance of the mixed-size batch, in launch order."""
    out = []
    for n in sizes:
        out += [_gemm(n), _gemm3(n), _gemv_family("gemv", n), _gemv_family("gemv_t", n),
                _gemv_family("gemv_pair", n), _conv2d(n), _colstats(n), _corr(n)]
    out.append(_conv3d(conv3d_size))
    return out


def precision_instances(sizes=SIZES):
    """The reduced-precision contractions: GEMM in BF16 and split BF16 at every size,
    by both kernels (what their variants are tuned on)."""
    return [_gemm(n, p, prep) for prep in (True, False) for p in ("bf16", "split") for n in sizes]


def corr_precision_instances(sizes=SIZES):
    """The correlation in BF16 and split BF16 at every size (what the reduced-precision
    rank-k variants are tuned on)."""
    return [_corr(n, p) for p in ("bf16", "split") for n in sizes]


def config_instances():
    """The chained product in three precisions at 2048 and the correlation at 2048 in
    FP32, split BF16 and BF16: the precision comparison workloads."""
    return [_gemm3(2048, p) for p in ("fp32", "bf16", "split")] + \
           [_corr(2048, p) for p in ("fp32", "split", "bf16")]


# ---- the next rows: COVAR, SYRK, SYR2K, GESUMMV, MVT (accumulate form), FDTD-2D ----
NEXT_WORKLOAD = 8


def _covar(n):
    def make(dev, copies):
        X, _ = synth.corr_inputs(n, workload=NEXT_WORKLOAD)
        return dict(X=_copies(_g(X, dev), copies), C=torch.empty((n, n), device=dev),
                    mu=torch.empty(n, device=dev),
                    ws=torch.empty(ctx_ws("covar", (n, n)), dtype=torch.uint8, device=dev))

    def run(ctx, s, i, stream):
        ctx.covar(s["X"][i], C=s["C"], mean=s["mu"], ws=s["ws"], stream=stream)

    fl = 2.0 * n * n + n * (n + 1) / 2 * 2.0 * n
    return Instance(f"covar/{n}", "covar", ("colstats", "syrk_f32"), n, fl, 4.0 * (2 * n * n + n),
                    "mfma", make, run, 8 * n * n)


def _rankk(n, two):
    def make(dev, copies):
        A = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 0), (n, n)), dev)
        B = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 1), (n, n)), dev)
        C = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 2), (n, n)), dev)
        return dict(A=_copies(A, copies), B=_copies(B, copies), C=_copies(C, copies))

    def run(ctx, s, i, stream):
        if two:
            ctx.syr2k(s["A"][i], s["B"][i], s["C"][i], 1.5, 1.2, stream=stream)
        else:
            ctx.syrk(s["A"][i], s["C"][i], 1.5, 1.2, stream=stream)

    fl = (2.0 if two else 1.0) * n * (n + 1) / 2 * 2.0 * n + 3.0 * n * n
    by = 4.0 * ((3 if two else 2) * n * n + n * n)
    op = "syr2k" if two else "syrk"
    return Instance(f"{op}/{n}", op, ("rankk",), n, fl, by, "mfma", make, run, (16 if two else 12) * n * n)


def _gesummv(n):
    def make(dev, copies):
        A = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 0), (n, n)), dev)
        B = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 1), (n, n)), dev)
        x = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 4), (n,)), dev)
        return dict(A=_copies(A, copies), B=_copies(B, copies), x=x, y=torch.empty(n, device=dev))

    def run(ctx, s, i, stream):
        ctx.gesummv(s["A"][i], s["B"][i], s["x"], 1.5, 1.2, y=s["y"], stream=stream)

    return Instance(f"gesummv/{n}", "gesummv", ("gesummv",), n, 4.0 * n * n + 3.0 * n,
                    4.0 * (2 * n * n + 2 * n), "hbm", make, run, 8 * n * n)


def _mvt(n):
    def make(dev, copies):
        A = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 0), (n, n)), dev)
        vs = [_g(synth.uniform(synth.seed(NEXT_WORKLOAD, 4 + j), (n,)), dev) for j in range(4)]
        return dict(A=_copies(A, copies), y1=vs[0], y2=vs[1], x1=vs[2], x2=vs[3],
                    ws=torch.empty(ctx_ws("mvt", (n,)), dtype=torch.uint8, device=dev))

    def run(ctx, s, i, stream):
        ctx.mvt(s["A"][i], s["y1"], s["y2"], s["x1"], s["x2"], ws=s["ws"], stream=stream)

    return Instance(f"mvt/{n}", "mvt", ("gemv_pair", "gesummv"), n, 4.0 * n * n + 2.0 * n,
                    4.0 * (n * n + 6 * n), "hbm", make, run, 4 * n * n)


def _fdtd2d(n, steps=10):
    def make(dev, copies):
        fict = _g(synth.uniform(synth.seed(NEXT_WORKLOAD, 7), (steps,)), dev)
        f = [_g(synth.uniform(synth.seed(NEXT_WORKLOAD, 10 + j), (n, n), -1.0, 1.0), dev) for j in range(3)]
        return dict(fict=fict, ex=_copies(f[0], copies), ey=_copies(f[1], copies), hz=_copies(f[2], copies))

    def run(ctx, s, i, stream):
        ctx.fdtd2d(s["fict"], s["ex"][i], s["ey"][i], s["hz"][i], stream=stream)

    # per step and cell: E update reads hz, ey, ex and writes ey, ex; H update reads
    # ex, ey, hz and writes hz (neighbour reads come from cache): 9 floats.  When the
    # three fields fit in the 256 MB Infinity Cache they stay there across the steps
    # of a call, and the bound is that cache's bandwidth, not HBM's
    bound = "infinity_cache" if 12 * n * n <= (256 << 20) else "hbm"
    return Instance(f"fdtd2d/{n}x{steps}", "fdtd2d", ("fdtd",), n, 11.0 * n * n * steps,
                    36.0 * n * n * steps, bound, make, run, 12 * n * n)


def next_tuning_instances(sizes=SIZES):
    """What the next rows' kernel families are tuned on: SYRK (family rankk),
    GESUMMV (family gesummv) and FDTD-2D, 10 steps (family fdtd), at every size."""
    return [_rankk(n, False) for n in sizes] + [_gesummv(n) for n in sizes] + [_fdtd2d(n) for n in sizes]


def next_instances():
    """The next rows of the method at their largest sizes."""
    return [_covar(2048), _covar(4096), _rankk(4096, False), _rankk(4096, True), _gesummv(4096), _mvt(4096),
            _fdtd2d(4096)]


TUNED_FAMILIES = ("gemm_f32", "gemv", "gemv_t", "gemv_pair", "conv2d", "conv3d", "colstats", "syrk_f32")

# the operation each kernel family is timed on (the family's own; a family not
# listed is timed on the operation of the same name)
FAMILY_OP = {"gemm_f32": "gemm", "syrk_f32": "corr", "gemm_bf16_ws": "gemm_bf16ws", "gemm_split_ws": "gemm_splitws",
             "syrk_bf16": "corr_bf16", "syrk_split": "corr_split", "rankk": "syrk", "fdtd": "fdtd2d"}


def family_instances(family, sizes=SIZES):
    """The instances a kernel family is timed on: its own operation at `sizes`."""
    op = FAMILY_OP.get(family, family)
    return [i for i in batch_instances(tuple(sizes)) + precision_instances(tuple(sizes))
            + corr_precision_instances(tuple(sizes)) + next_tuning_instances(tuple(sizes)) if i.op == op]
