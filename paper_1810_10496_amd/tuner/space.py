"""The variant space: knob domains per kernel family and the seeded sampler.

A variant is (knobs, pipeline, llc flags).  Knobs are the kernel source's
compile-time parameters (tile shape, wavefronts per block, vector width,
unroll, LDS staging, loop/raster order); the pipeline is an ``opt -passes=``
string, either a standard level or a phase order drawn from the pass pool.

As in the paper's exploration (Sec. 3: one set of random phase orders used
for every kernel), the pipeline sample is one seeded list shared by all
families; the knob sample is seeded per family.  Constraints keep every
sampled variant buildable within the hardware limits (LDS per block,
registers for accumulators, threads per block).
"""
from __future__ import annotations

import random
from dataclasses import dataclass

from .. import codegen

# ------------------------------------------------------------------- knobs --

DOMAINS = {
    "gemm_f32": dict(BM=[16, 32, 64, 128, 256], BN=[16, 32, 64, 128, 256], BK=[16, 32],
                     WAVES_M=[1, 2, 4], WAVES_N=[1, 2, 4], VEC=[1, 2, 4], UNROLL=[1, 2],
                     USE_LDS=[0, 1, 2], ORDER=[0, 1, 2, 3]),
    "gemv": dict(ROWS=[1, 2, 4], WAVES=[1, 2, 4, 8], VEC=[1, 2, 4], UNROLL=[1, 2, 4, 8],
                 USE_LDS=[0, 1], ORDER=[0]),
    "gemv_t": dict(ROWS=[16, 32, 64, 128, 256], WAVES=[1, 2, 4, 8], VEC=[1, 2, 4], UNROLL=[1, 2, 4, 8, 16],
                   ORDER=[0, 1]),
    "gemv_pair": dict(ROWS=[16, 32, 64, 128, 256], WAVES=[1, 2, 4, 8], VEC=[1, 2, 4], UNROLL=[4, 8, 16, 32],
                      ORDER=[0, 1]),
    "conv2d": dict(VEC=[1, 2, 4], TX=[16, 32, 64, 128], TY=[1, 2, 4, 8, 16], ROWS=[1, 2, 4, 8, 16],
                   UNROLL=[1, 2, 4], USE_LDS=[0, 1], ORDER=[0, 1, 2]),
    "conv3d": dict(VEC=[1, 2, 4], TX=[16, 32, 64, 128], TY=[1, 2, 4, 8, 16], ROWS=[1, 2, 4, 8, 16, 32],
                   UNROLL=[1, 2], USE_LDS=[0, 1, 2], ORDER=[0, 1, 2], YR=[1, 2, 4, 8]),
    "colstats": dict(VEC=[1, 2, 4], WAVES=[1, 2, 4, 8], ROWS=[16, 32, 64, 128, 256], ORDER=[0, 1]),
    "syrk_f32": dict(BT=[32, 48, 64, 96, 128], BK=[16, 32], WAVES_M=[1, 2, 4], WAVES_N=[1, 2, 4],
                     VEC=[1, 2, 4], STAGES=[1, 2], ORDER=[0, 2]),
}
# Knobs the kernels gained after the exploration sample was drawn: the random sample
# leaves them at their defaults (so it, and the table measured from it, stay as they
# were); `tuner refine` times structured grids over them against the finished table.
#   FUSE: one launch for the transposed matvec, the pair and the column statistics
#   PF:   planes fetched ahead by the staged 3D stencil
#   EPI:  the prepared bf16 GEMM's epilogue can write the next product's prepared operand
#   MF, LDS_PAD, FC: the FP32 GEMM's MFMA block (16 or 32), LDS row padding, fragments
#   read in chunks of four k (deep k-steps; BK 64, also refine-only, may use the whole LDS);
#   IL: the interleaved k loop of full interior tiles (two LDS stages)
REFINE_ONLY = {
    "gemm_f32": dict(MF=[16, 32], LDS_PAD=[4, 8], FC=[0, 4], IL=[0, 1, 2], DK=[0, 1]),
    "gemv": dict(NTL=[0, 1]),
    "gemv_t": dict(FUSE=[0, 1], NTL=[0, 1]),
    "gemv_pair": dict(FUSE=[0, 1], NTL=[0, 1]),
    "colstats": dict(FUSE=[0, 1], NTL=[0, 1], MG=[0, 1]),
    "gesummv": dict(NTL=[0, 1]),
    "conv2d": dict(NTL=[0, 1]),
    "conv3d": dict(PF=[1, 2], NTL=[0, 1]),
    "gemm_bf16_ws": dict(EPI=[0, 1]),
    "gemm_split_ws": dict(EPI=[0, 1]),
    "syrk_f32": dict(IL=[0, 1, 2, 3]),
}

# the reduced-precision contractions: bf16 fragments need BK in multiples of 32
for _fam in ("gemm_bf16", "gemm_split"):
    DOMAINS[_fam] = dict(BM=[64, 128, 256], BN=[64, 128, 256], BK=[32, 64], WAVES_M=[1, 2, 4], WAVES_N=[1, 2, 4],
                         VEC=[1, 2, 4], STAGES=[1, 2], ORDER=[0, 1, 2, 3])

for _fam in ("gemm_bf16_ws", "gemm_split_ws"):
    DOMAINS[_fam] = dict(BM=[64, 128, 256], BN=[64, 128, 256], BK=[32, 64], WAVES_M=[1, 2, 4],
                         WAVES_N=[1, 2, 4], ORDER=[0, 1, 2, 3], LDS_PAD=[8, 16, 24],
                         PIPE=[0, 1, 2], DSTAGES=[2, 3, 4], SCHED=[0, 1])
# the next rows' kernels: SYRK / SYR2K, GESUMMV (+ MVT's accumulating reduce), FDTD-2D
DOMAINS["rankk"] = dict(BT=[32, 64, 128], BK=[16, 32], WAVES_M=[1, 2, 4], WAVES_N=[1, 2, 4], VEC=[1, 2, 4],
                        UNROLL=[1, 2])
DOMAINS["gesummv"] = dict(ROWS=[1, 2, 4], WAVES=[1, 2, 4, 8], VEC=[1, 2, 4], UNROLL=[1, 2, 4, 8])
DOMAINS["fdtd"] = dict(VEC=[1, 2, 4], TX=[16, 32, 64, 128], TY=[1, 2, 4, 8, 16])
# the correlation's rank-k product in bf16 / split: the same kernel in its
# lower-triangle form (square tiles, triangle rasters 0 and 2).  Widths 96 and 192
# put the triangle's tile count just under a multiple of the 256 CUs at 2048 and
# 4096 (253 tiles either way), where the powers of two leave CUs idle
for _fam in ("syrk_bf16", "syrk_split"):
    DOMAINS[_fam] = dict(BM=[64, 96, 128, 192, 256], BN=[64, 96, 128, 192, 256], BK=[32, 64], WAVES_M=[1, 2, 4],
                         WAVES_N=[1, 2, 4], ORDER=[0, 2], LDS_PAD=[8, 16, 24],
                         PIPE=[0, 1, 2], DSTAGES=[2, 3, 4], SCHED=[0, 1])

LDS_LIMIT = 64 * 1024
LDS_LIMIT_GFX950 = 160 * 1024    # the whole LDS of a CU, usable by one workgroup


def valid(family: str, k: dict) -> bool:
    """Hardware and kernel constraints of one knob setting."""
    if family in ("gemm_bf16", "gemm_split"):
        wtm, wtn = k["BM"] // k["WAVES_M"], k["BN"] // k["WAVES_N"]
        if k["BM"] % k["WAVES_M"] or k["BN"] % k["WAVES_N"] or wtm % 16 or wtn % 16:
            return False
        if (wtm // 16) * (wtn // 16) > 32:            # accumulator registers per lane <= 128
            return False
        planes = 2 if family == "gemm_split" else 1
        lds = k["STAGES"] * planes * (k["BM"] + k["BN"]) * (k["BK"] + 8) * 2
        return lds <= LDS_LIMIT_GFX950 and 64 * k["WAVES_M"] * k["WAVES_N"] <= 1024
    if family in ("syrk_bf16", "syrk_split"):
        if k["BM"] != k["BN"]:
            return False
        return valid("gemm_bf16_ws" if family == "syrk_bf16" else "gemm_split_ws", k)
    if family in ("gemm_bf16_ws", "gemm_split_ws"):
        wtm, wtn = k["BM"] // k["WAVES_M"], k["BN"] // k["WAVES_N"]
        if k["BM"] % k["WAVES_M"] or k["BN"] % k["WAVES_N"] or wtm % 16 or wtn % 16:
            return False
        if (wtm // 16) * (wtn // 16) > 64:            # accumulator registers per lane <= 256
            return False
        nt = 64 * k["WAVES_M"] * k["WAVES_N"]
        if nt > 1024:
            return False
        planes = 2 if family == "gemm_split_ws" else 1
        pipe, cpr = k["PIPE"], k["BK"] // 8
        if pipe == 0:
            # register-staged tiles: the stage count and scheduling fence do not
            # apply, so only one setting of each is a distinct variant
            if k["DSTAGES"] != 2 or k["SCHED"] != 0:
                return False
            lds = 2 * planes * (k["BM"] + k["BN"]) * (k["BK"] + k["LDS_PAD"]) * 2
            return lds <= LDS_LIMIT_GFX950
        # direct-to-LDS pipelines: unpadded swizzled tiles, whole chunks per thread
        if k["LDS_PAD"] != 8 or k["DSTAGES"] not in ((2, 3) if pipe == 1 else (3, 4)):
            return False
        if pipe == 3 and (nt // 64) % 2:              # ping-pong: two equal wave groups
            return False
        if (k["BM"] * cpr) % nt or (k["BN"] * cpr) % nt:
            return False
        if planes * (k["BM"] + k["BN"]) * cpr // nt > 63:
            return False
        if k["DSTAGES"] * planes * (k["BM"] + k["BN"]) * k["BK"] * 2 > LDS_LIMIT_GFX950:
            return False
        if pipe in (2, 3):
            # accumulators plus the fragments held at once (PIPE 2: two k-steps'
            # sets; PIPE 3: every k-step of a tile) within the registers a wave
            # gets when the workgroup's waves share the four SIMDs
            fm, fn = wtm // 16, wtn // 16
            sets = 2 if pipe == 2 else k["BK"] // 32
            regs = 4 * fm * fn + sets * 4 * planes * (fm + fn) + 24
            budget = 512 // max(1, nt // 256)
            return regs <= min(budget, 512)
        return True
    if family == "gemm_f32":
        wtm, wtn = k["BM"] // k["WAVES_M"], k["BN"] // k["WAVES_N"]
        blk = k.get("MF", 16)
        if k["BM"] % k["WAVES_M"] or k["BN"] % k["WAVES_N"] or wtm % blk or wtn % blk:
            return False
        # accumulator registers per lane: <= 128, or <= 256 for the 32x32 blocks (AGPRs)
        if wtm * wtn // 64 > (256 if blk == 32 else 128):
            return False
        if k["BN"] % k["VEC"] or k["BK"] % k["VEC"] or (blk == 32 and k["BK"] % 8):
            return False
        stages = 2 if k["USE_LDS"] == 2 else 1
        lds = stages * (k["BM"] + k["BN"]) * (k["BK"] + k.get("LDS_PAD", 4)) * 4 if k["USE_LDS"] else 0
        if k.get("FC", 0) and ((k["BK"] // (64 // blk)) % 4 or blk != 16 and blk != 32):
            return False
        if k.get("DK", 0) and k["USE_LDS"] != 0:
            return False
        if k["UNROLL"] > 2 and not k.get("DK", 0):
            return False                     # deep unrolls only for the branch-free direct loads
        if k.get("IL", 0):
            nt = 64 * k["WAVES_M"] * k["WAVES_N"]
            if (k["USE_LDS"] != 2 or k.get("FC", 0) or k["VEC"] != 4 or (k["BM"] * k["BK"] // 4) % nt
                    or (k["BK"] * k["BN"] // 4) % nt):
                return False
        limit = LDS_LIMIT_GFX950 if k["BK"] == 64 or k.get("IL", 0) else LDS_LIMIT
        return lds <= limit and 64 * k["WAVES_M"] * k["WAVES_N"] <= 1024
    if family == "syrk_f32":
        wtm, wtn = k["BT"] // k["WAVES_M"], k["BT"] // k["WAVES_N"]
        if k["BT"] % k["WAVES_M"] or k["BT"] % k["WAVES_N"] or wtm % 16 or wtn % 16:
            return False
        if (wtm // 16) * (wtn // 16) > 32 or k["BT"] % k["VEC"]:
            return False
        ldr = k["BT"] + (16 if k["BT"] % 32 == 0 else 32)
        if k.get("IL", 0) and (k["STAGES"] != 2 or k["VEC"] != 4 or (k["BK"] * k["BT"] // 4) % (64 * k["WAVES_M"] * k["WAVES_N"])):
            return False
        return k["STAGES"] * 2 * k["BK"] * ldr * 4 + 16 * k["BT"] <= (LDS_LIMIT_GFX950 if k.get("IL", 0) else LDS_LIMIT)
    if family == "rankk":
        wtm, wtn = k["BT"] // k["WAVES_M"], k["BT"] // k["WAVES_N"]
        if k["BT"] % k["WAVES_M"] or k["BT"] % k["WAVES_N"] or wtm % 16 or wtn % 16:
            return False
        if (wtm // 16) * (wtn // 16) > 32 or k["BK"] % k["VEC"]:
            return False
        return 4 * k["BT"] * (k["BK"] + 4) * 4 <= LDS_LIMIT_GFX950
    if family == "gesummv":
        return True
    if family == "fdtd":
        nt = k["TX"] * k["TY"]
        return nt % 64 == 0 and nt <= 1024
    if family == "gemv":
        return True
    if family in ("gemv_t", "gemv_pair"):
        if k.get("FUSE", 0):
            # one launch: the wavefronts share the block's columns and split its rows
            rpw = k["ROWS"] // k["WAVES"]
            return (k["ROWS"] % k["WAVES"] == 0 and rpw % k["UNROLL"] == 0
                    and k["UNROLL"] * k["VEC"] <= 128)
        return k["ROWS"] % k["UNROLL"] == 0 and k["UNROLL"] * k["VEC"] <= 128
    if family in ("conv2d", "conv3d"):
        nt = k["TX"] * k["TY"]
        if nt % 64 or nt > 1024:
            return False
        if family == "conv2d" and k["USE_LDS"]:
            return (k["TY"] * k["ROWS"] + 2) * (k["TX"] * k["VEC"] + 4) * 4 <= LDS_LIMIT
        if family == "conv3d" and k["USE_LDS"] == 2:
            return k["TY"] * k["YR"] <= 64 and 4 * (k["TY"] * k["YR"] + 2) * (k["TX"] * k["VEC"] + 8) * 4 <= LDS_LIMIT_GFX950
        if family == "conv3d" and k["USE_LDS"]:
            return 3 * (k["TY"] + 2) * (k["TX"] * k["VEC"] + 4) * 4 <= LDS_LIMIT
        return True
    if family == "colstats":
        if k.get("MG", 0) and k.get("FUSE", 0):
            return False                     # the one-launch form has no separate merge
        rpw = -(-k["ROWS"] // k["WAVES"])
        lds = (3 * k["WAVES"] + 1) * 64 * k["VEC"] * 4
        return rpw * k["VEC"] <= 128 and lds <= LDS_LIMIT
    raise KeyError(family)


def sample_knobs(family: str, count: int, seed: int) -> list[dict]:
    """`count` valid knob settings (with repetition allowed) drawn uniformly."""
    dom = DOMAINS[family]
    rng = random.Random(f"{seed}:{family}")
    out = []
    while len(out) < count:
        k = {name: rng.choice(vals) for name, vals in dom.items()}
        if valid(family, k):
            out.append(k)
    return out


def default_knobs(family: str) -> dict:
    return dict(codegen.FAMILIES[family].defaults)


# --------------------------------------------------------------- pipelines --

STANDARD = ["default<O3>", "default<O2>", "default<O1>", "default<Os>", "default<Oz>"]

# flags of the standard pipelines' own passes (cost models) and of the AMDGPU
# back end (machine scheduler strategy); None = the pass's default
OPT_FLAG_CHOICES = {
    "-unroll-threshold": [None, 150, 300, 600, 1200],
    "-inline-threshold": [None, 500, 1000],
    "-unroll-allow-partial": [None, True],
    "-unroll-runtime": [None, True],
}
LLC_FLAG_CHOICES = {
    "-misched": [None, "gcn-max-occupancy", "gcn-max-ilp", "gcn-max-memory-clause"],
    "-amdgpu-schedule-metric-bias": [None, 0, 50, 100],
}


class RandomOrdersDisabled(RuntimeError):
    pass


@dataclass
class PipelineMix:
    """Shares of the knob exploration's pipeline sample.

    The knob exploration pairs each knob draw with a standard pipeline (some
    with flags of their passes); its sample, and the tuning table measured
    from it, stay fixed.  Random phase orders (the paper's Sec. 3 kind, alone
    or after -O3) are explored on fixed knobs by `tuner.orders`, where every
    code object passes the gate of `tuner.gate` before it runs.  Mixing them
    into this sample needs `allow_random_orders=True`."""
    o3: float = 0.45              # the standard -O3 pipeline, default flags
    other_levels: float = 0.15    # -O1/-O2/-Os/-Oz
    flagged: float = 0.40         # -O3 with sampled opt/llc flags
    random_order: float = 0.0     # a random phase order alone
    o3_suffix: float = 0.0        # -O3 followed by a random phase order
    max_len: int = 128
    max_suffix: int = 16


def _flags(rng, choices, fmt):
    out = []
    for name, vals in choices.items():
        v = rng.choice(vals)
        if v is None:
            continue
        out.append(name if v is True else f"{name}={v}")
    return tuple(out)


def sample_pipelines(pool: list[str], count: int, seed: int, mix: PipelineMix = PipelineMix(),
                     allow_random_orders: bool = False) -> list[tuple]:
    """One seeded list of (pipeline, opt flags, llc flags), shared by every family.

    `pool` holds wrapped pass strings (e.g. "function(gvn)"); a random phase
    order draws 1..max_len of them uniformly with repetition."""
    if (mix.random_order > 0 or mix.o3_suffix > 0) and not allow_random_orders:
        raise RandomOrdersDisabled("random phase orders are not part of the knob exploration's sample")
    rng = random.Random(f"{seed}:pipelines")
    out = []
    edges = [mix.o3, mix.other_levels, mix.flagged, mix.random_order, mix.o3_suffix]
    total = sum(edges)
    for _ in range(count):
        u = rng.random() * total
        if u < edges[0]:
            out.append(("default<O3>", (), ("-O3",)))
        elif u < sum(edges[:2]):
            out.append((rng.choice(STANDARD[1:]), (), ("-O3",)))
        elif u < sum(edges[:3]):
            of = _flags(rng, OPT_FLAG_CHOICES, "opt")
            lf = ("-O3",) + _flags(rng, LLC_FLAG_CHOICES, "llc")
            out.append(("default<O3>", of, lf))
        elif u < sum(edges[:4]) and pool:
            n = rng.randint(1, mix.max_len)
            out.append((",".join(rng.choice(pool) for _ in range(n)), (), ("-O3",)))
        elif pool:
            n = rng.randint(1, mix.max_suffix)
            out.append(("default<O3>," + ",".join(rng.choice(pool) for _ in range(n)), (), ("-O3",)))
        else:
            out.append(("default<O3>", (), ("-O3",)))
    return out


@dataclass
class Variant:
    family: str
    knobs: dict
    pipeline: str
    llc_flags: tuple = ("-O3",)
    opt_flags: tuple = ()

    def key(self) -> str:
        ks = ",".join(f"{k}={self.knobs[k]}" for k in sorted(self.knobs))
        return f"{self.family}|{ks}|{' '.join(self.opt_flags)}|{self.pipeline}|{' '.join(self.llc_flags)}"

    def to_json(self) -> dict:
        return dict(family=self.family, knobs=dict(self.knobs), pipeline=self.pipeline,
                    llc_flags=list(self.llc_flags), opt_flags=list(self.opt_flags))

    @staticmethod
    def from_json(d: dict) -> "Variant":
        return Variant(d["family"], dict(d["knobs"]), d["pipeline"], tuple(d.get("llc_flags", ["-O3"])),
                       tuple(d.get("opt_flags", [])))


def sample_variants(family: str, pool: list[str], count: int = 500, seed: int = 5500,
                    mix: PipelineMix = PipelineMix(), allow_random_orders: bool = False) -> list[Variant]:
    """The family's exploration sample: variant i pairs knob draw i with pipeline i."""
    knobs = sample_knobs(family, count, seed)
    pipes = sample_pipelines(pool, count, seed, mix, allow_random_orders)
    return [Variant(family, k, p, lf, of) for k, (p, of, lf) in zip(knobs, pipes)]


def default_variant(family: str) -> Variant:
    return Variant(family, default_knobs(family), codegen.DEFAULT_PIPELINE)


def transfer(source: Variant, target_family: str) -> Variant | None:
    """Carry a variant of one family over to another (feature-based reuse).

    The pipeline transfers as is; knobs the two families share by name take
    the source's values when the result is valid for the target, the rest
    keep the target's defaults."""
    k = default_knobs(target_family)
    for name, v in source.knobs.items():
        if name in k and v in DOMAINS[target_family].get(name, [v]):
            trial = dict(k)
            trial[name] = v
            if valid(target_family, trial):
                k = trial
    return Variant(target_family, k, source.pipeline, source.llc_flags, source.opt_flags)
