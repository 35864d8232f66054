"""GPU evaluation worker for the tuner.

One worker process owns the GPU context for one kernel family.  The explorer
sends it requests as JSON lines on stdin and reads one JSON line back per
request; a crash or a hang costs only this process (the explorer kills and
restarts it and records the candidate as crashed or timed out).

Validation (the paper validates each phase order against the sequential
version on small inputs, Sec. 2.4): a candidate runs the family's small
validation cases and its outputs are compared with those of the family's
built-in default variant, whose own results the test suite pins to the FP64
oracle.  Cases with small-integer inputs must match bitwise (exact
arithmetic); seeded real-valued cases must agree within the FP32 bar.  Every
output buffer is filled with NaN first, so unwritten elements fail.

Timing: each of the family's batch instances is captured as graphs of `reps`
and 2*`reps` launches on rotating operand copies; the difference of their
replay times over `reps` is the time per launch, reported per size (the
median of `replays` replays, free of the graph launch cost).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import traceback

import numpy as np
import torch

from .. import api, synth, workloads as W
from ..timing import per_launch_ms
from . import gate

DEV = "cuda:0"
ROTATE_BYTES = 640 << 20
CACHE_BYTES = 512 << 20       # rotations at least this large stream from HBM (256 MB Infinity Cache)
PEAK_HBM = 8.0e12             # B/s
PEAK_FP32 = 157.3e12          # flop/s
PEAK_BF16 = 2516.6e12         # flop/s, dense


class Implausible(RuntimeError):
    """A measured time faster than the roofline allows."""
TAPS2 = np.array(synth.CONV2D_TAPS, np.float32)


def g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def nan_like(t):
    return torch.full_like(t, float("nan"))


# -------------------------------------------------------------- validation cases --
# each case: (name, inputs builder(seed) -> dict, run(ctx, st) -> list of output tensors, exact, rtol, atol)

def _gemm_case(M, N, K, ints=False, prec="fp32", ws=None):
    def build(seed):
        if ints:
            A = synth.small_ints(900 + seed, (M, K))
            B = synth.small_ints(901 + seed, (K, N))
            C = synth.small_ints(902 + seed, (M, N))
            al, be = 2.0, 0.5
        else:
            A = synth.uniform(910 + seed, (M, K))
            B = synth.uniform(911 + seed, (K, N))
            C = synth.uniform(912 + seed, (M, N))
            al, be = 1.5, 1.2
        return dict(A=g(A), B=g(B), C0=g(C), C=g(C), al=al, be=be)

    def run(ctx, st):
        st["C"].copy_(st["C0"])
        ctx.gemm(st["A"], st["B"], st["C"], st["al"], st["be"], prec=prec, ws=ws)
        return [st["C"]]
    # candidates are compared with the default variant of the same precision: the
    # operands are rounded identically, only the order of the FP32 sums differs
    return (f"gemm{M}x{N}x{K}{'i' if ints else ''}", build, run, ints, 1e-4, 0.0)


def _gemv_case(op, M, N, ints=False):
    def build(seed):
        if ints:
            A = synth.small_ints(920 + seed, (M, N))
            x = synth.small_ints(921 + seed, (N,))
            z = synth.small_ints(922 + seed, (M,))
        else:
            A = synth.uniform(930 + seed, (M, N))
            x = synth.uniform(931 + seed, (N,))
            z = synth.uniform(932 + seed, (M,))
        return dict(A=g(A), x=g(x), z=g(z), y1=torch.empty(M, device=DEV), y2=torch.empty(N, device=DEV))

    def run(ctx, st):
        st["y1"].fill_(float("nan"))
        st["y2"].fill_(float("nan"))
        if op == "gemv":
            ctx.gemv(st["A"], st["x"], st["y1"])
            return [st["y1"]]
        if op == "gemv_t":
            ctx.gemv_t(st["A"], st["z"], st["y2"])
            return [st["y2"]]
        ctx.gemv_pair(st["A"], st["x"], st["z"], st["y1"], st["y2"])
        return [st["y1"], st["y2"]]
    return (f"{op}{M}x{N}{'i' if ints else ''}", build, run, ints, 1e-4, 0.0)


def _conv2d_case(H, W_, ints=False):
    def build(seed):
        if ints:
            grid = synth.small_ints(940 + seed, (H, W_), -8, 8)
            taps = (synth.small_ints(941 + seed, (9,), -8, 8) / 8).astype(np.float32)
        else:
            grid = synth.uniform(942 + seed, (H, W_))
            taps = TAPS2
        return dict(inp=g(grid), out=torch.empty((H, W_), device=DEV), taps=taps)

    def run(ctx, st):
        st["out"].fill_(float("nan"))
        ctx.conv2d(st["inp"], st["taps"], out=st["out"])
        return [st["out"]]
    # signed taps: compare against the reference's magnitude scale (atol ~ tol * typical |x|)
    return (f"conv2d{H}x{W_}{'i' if ints else ''}", build, run, ints, 1e-4, 1e-5)


def _conv3d_case(D, H, W_):
    def build(seed):
        vol = synth.uniform(950 + seed, (D, H, W_))
        taps = synth.uniform(951 + seed, (27,), -1, 1)
        return dict(inp=g(vol), out=torch.empty((D, H, W_), device=DEV), taps=taps)

    def run(ctx, st):
        st["out"].fill_(float("nan"))
        ctx.conv3d(st["inp"], st["taps"], out=st["out"])
        return [st["out"]]
    return (f"conv3d{D}x{H}x{W_}", build, run, False, 1e-4, 1e-5)


def _colstats_case(n, m):
    def build(seed):
        X, eps = synth.corr_inputs(n, m, workload=60 + seed)
        return dict(X=g(X), eps=float(eps), mu=torch.empty(m, device=DEV), sd=torch.empty(m, device=DEV))

    def run(ctx, st):
        st["mu"].fill_(float("nan"))
        st["sd"].fill_(float("nan"))
        ctx.colstats(st["X"], st["eps"], st["mu"], st["sd"])
        return [st["mu"], st["sd"]]
    return (f"colstats{n}x{m}", build, run, False, 1e-5, 0.0)


def _corr_case(n, m, prec="fp32"):
    def build(seed):
        X, eps = synth.corr_inputs(n, m, workload=70 + seed)
        return dict(X=g(X), eps=float(eps), R=torch.empty((m, m), device=DEV))

    def run(ctx, st):
        st["R"].fill_(float("nan"))
        R, _, _ = ctx.corr(st["X"], st["eps"], prec=prec, R=st["R"])
        return [R]
    # |R| <= 1: absolute bars (bf16 rounding of z gives errors near 1e-3 of |z|^2)
    atol = {"fp32": 1e-4, "bf16": 2e-2, "split": 1e-5}[prec]
    return (f"corr{n}x{m}{prec}", build, run, False, 0.0, atol)


def _rankk_case(N, K, two):
    def build(seed):
        A = synth.uniform(960 + seed, (N, K), -1, 1)
        B = synth.uniform(961 + seed, (N, K), -1, 1)
        C = synth.uniform(962 + seed, (N, N), -1, 1)
        return dict(A=g(A), B=g(B), C0=g(C), C=g(C))

    def run(ctx, st):
        st["C"].copy_(st["C0"])
        if two:
            ctx.syr2k(st["A"], st["B"], st["C"], 1.5, -0.75)
        else:
            ctx.syrk(st["A"], st["C"], 1.5, -0.75)
        return [st["C"]]
    # signed operands: an absolute bar on the scale of the largest output
    return (f"{'syr2k' if two else 'syrk'}{N}x{K}", build, run, False, 1e-4, 1e-5)


def _gesummv_case(N):
    def build(seed):
        A = synth.uniform(970 + seed, (N, N))
        B = synth.uniform(971 + seed, (N, N))
        x = synth.uniform(972 + seed, (N,))
        return dict(A=g(A), B=g(B), x=g(x), y=torch.empty(N, device=DEV))

    def run(ctx, st):
        st["y"].fill_(float("nan"))
        return [ctx.gesummv(st["A"], st["B"], st["x"], 1.5, 1.2, y=st["y"])]
    return (f"gesummv{N}", build, run, False, 1e-4, 0.0)


def _fdtd_case(NX, NY, steps=3):
    def build(seed):
        f = [synth.uniform(980 + 3 * seed + j, (NX, NY), -1, 1) for j in range(3)]
        fict = synth.uniform(979 + seed, (steps,))
        return dict(fict=g(fict), f0=[g(x) for x in f], f=[g(x) for x in f])

    def run(ctx, st):
        for d, s0 in zip(st["f"], st["f0"]):
            d.copy_(s0)
        ctx.fdtd2d(st["fict"], *st["f"])
        return list(st["f"])
    return (f"fdtd{NX}x{NY}", build, run, False, 1e-4, 1e-5)


def validation_cases(family):
    """Small cases per family: ragged shapes that exercise every tile edge, degenerate
    ones, exact small-integer ones, and shapes that are whole multiples of every tile
    width the family's knobs allow (so the paths without any edge run too; a miscompiled
    edge-free loop otherwise passes every ragged case)."""
    if family == "gemm_f32":
        return [_gemm_case(65, 33, 47), _gemm_case(128, 96, 200), _gemm_case(1, 1, 1), _gemm_case(61, 70, 90, True),
                _gemm_case(257, 129, 64), _gemm_case(512, 512, 256), _gemm_case(256, 256, 128, True)]
    if family in ("gemm_bf16", "gemm_split", "gemm_bf16_ws", "gemm_split_ws"):
        prec = "bf16" if family.startswith("gemm_bf16") else "split"
        ws = None if family.endswith("_ws") else False
        return [_gemm_case(65, 33, 47, prec=prec, ws=ws), _gemm_case(300, 200, 129, prec=prec, ws=ws),
                _gemm_case(1, 1, 1, prec=prec, ws=ws), _gemm_case(61, 70, 90, True, prec=prec, ws=ws),
                _gemm_case(257, 129, 64, prec=prec, ws=ws), _gemm_case(512, 512, 256, prec=prec, ws=ws)]
    if family in ("gemv", "gemv_t", "gemv_pair"):
        return [_gemv_case(family, 77, 130), _gemv_case(family, 1000, 257), _gemv_case(family, 3, 5),
                _gemv_case(family, 333, 515, True), _gemv_case(family, 512, 2048), _gemv_case(family, 1024, 512, True)]
    if family == "conv2d":
        return [_conv2d_case(67, 131), _conv2d_case(5, 6), _conv2d_case(257, 300), _conv2d_case(40, 70, True),
                _conv2d_case(512, 512)]
    if family == "conv3d":
        return [_conv3d_case(17, 33, 65), _conv3d_case(3, 3, 3), _conv3d_case(20, 40, 70), _conv3d_case(16, 128, 512)]
    if family == "colstats":
        return [_colstats_case(130, 70), _colstats_case(1000, 257), _colstats_case(2, 5), _colstats_case(1024, 1024)]
    if family == "syrk_f32":
        return [_corr_case(257, 129), _corr_case(130, 70), _corr_case(2, 3), _corr_case(300, 64), _corr_case(512, 384)]
    if family == "rankk":
        return [_rankk_case(65, 33, False), _rankk_case(130, 200, False), _rankk_case(1, 1, False),
                _rankk_case(97, 64, True), _rankk_case(200, 17, True), _rankk_case(384, 256, False),
                _rankk_case(256, 128, True)]
    if family == "gesummv":
        return [_gesummv_case(77), _gesummv_case(1000), _gesummv_case(3), _gesummv_case(2048)]
    if family == "fdtd":
        return [_fdtd_case(67, 131), _fdtd_case(5, 6), _fdtd_case(200, 257), _fdtd_case(512, 512)]
    if family in ("syrk_bf16", "syrk_split"):
        prec = "bf16" if family == "syrk_bf16" else "split"
        return [_corr_case(257, 129, prec), _corr_case(130, 70, prec), _corr_case(2, 3, prec),
                _corr_case(300, 200, prec), _corr_case(512, 384, prec)]
    raise KeyError(family)


def compare(out, ref, exact, rtol, atol):
    """Largest violation ratio (<= 1 passes); inf on NaN or shape mismatch."""
    worst = 0.0
    for o, r in zip(out, ref):
        o = o.detach().cpu().numpy().astype(np.float64)
        r = r.astype(np.float64)
        if o.shape != r.shape or not np.all(np.isfinite(o)):
            return math.inf
        if exact:
            if not np.array_equal(o, r):
                return math.inf
            continue
        bound = rtol * np.abs(r) + atol * max(1.0, float(np.max(np.abs(r))) if r.size else 1.0)
        d = np.abs(o - r)
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(bound > 0, d / np.where(bound > 0, bound, 1.0), np.where(d == 0, 0.0, np.inf))
        worst = max(worst, float(ratio.max()) if ratio.size else 0.0)
    return worst


class Worker:
    def __init__(self, family, sizes, reps):
        self.family = family
        self.ctx = api.context(0)
        self.stream = torch.cuda.Stream()
        self.reps = reps
        self.default_vid = self.ctx.variant_default(family)
        # the instances each family is timed on: its own operation at every size
        self.insts = W.family_instances(family, tuple(sizes))
        for inst in self.insts:
            copies = max(1, min(reps, math.ceil(ROTATE_BYTES / max(inst.footprint, 1))))
            inst.state = inst.make(torch.device(DEV), copies)
            inst.state["_copies"] = copies
        self.cases = validation_cases(family)
        self.refs = {}     # (case name, seed) -> list of numpy outputs from the default variant
        torch.cuda.synchronize()

    def _with(self, vid, fn):
        self.ctx.variant_select(self.family, vid)
        try:
            return fn()
        finally:
            self.ctx.variant_select(self.family, -1)

    def _ref(self, case, seed):
        key = (case[0], seed)
        if key not in self.refs:
            st = case[1](seed)
            outs = self._with(self.default_vid, lambda: case[2](self.ctx, st))
            torch.cuda.synchronize()
            self.refs[key] = ([o.detach().cpu().numpy().copy() for o in outs], st)
        return self.refs[key]

    def validate(self, vid, seeds):
        worst = 0.0
        for seed in seeds:
            for case in self.cases:
                if case[3] and seed != 0:
                    continue       # integer cases once
                ref, st = self._ref(case, seed)
                outs = self._with(vid, lambda: case[2](self.ctx, st))
                torch.cuda.synchronize()
                r = compare(outs, ref, case[3], case[4], case[5])
                worst = max(worst, r)
                if r > 1.0:
                    return worst, f"{case[0]} seed {seed}"
        return worst, ""

    def floor_ms(self, inst):
        """The fastest a correct launch of `inst` can be: its useful flops at the matrix
        peak of its precision, and, when its rotating operand copies exceed the Infinity
        Cache (so that every launch reads HBM), its algorithmic bytes at the HBM peak."""
        low = any(p in self.family for p in ("bf16", "split"))
        t = inst.flops / (PEAK_BF16 if low else PEAK_FP32)
        if inst.bound == "hbm" and inst.footprint * inst.state.get("_copies", 1) >= CACHE_BYTES:
            t = max(t, inst.bytes / PEAK_HBM)
        return t * 1e3

    def time(self, vid, sizes, replays, cutoff):
        """ms per launch at each size; stops early when a size runs `cutoff` x slower
        than the given default times (then larger sizes are not timed).  A time below
        the size's roofline floor cannot come from code that did all the work: it raises
        Implausible (validation on small inputs cannot see every size's paths)."""
        out = {}
        for inst in self.insts:
            if sizes and inst.size not in sizes:
                continue
            self.ctx.variant_select(self.family, vid)
            try:
                t = per_launch_ms(self.ctx, self.stream,
                                  lambda i: inst.run(self.ctx, inst.state, i % inst.state["_copies"], self.stream),
                                  self.reps, replays)
            finally:
                self.ctx.variant_select(self.family, -1)
            out[str(inst.size)] = t
            floor = self.floor_ms(inst)
            if t < 0.95 * floor:
                raise Implausible(f"{inst.name}: {t * 1e3:.2f} us per launch, below its roofline floor "
                                  f"{floor * 1e3:.2f} us")
            lim = cutoff.get(str(inst.size)) if cutoff else None
            if lim is not None and t > lim:
                break
        return out

    def handle(self, req):
        op = req.get("op")
        if op == "eval":
            code = req.get("code")
            vid = self.default_vid
            loaded = False
            if code != "default":
                reason = gate.check_file(code)
                if reason:
                    return dict(status="gated", detail=reason[:300])
                try:
                    with open(code, "rb") as f:
                        vid = self.ctx.variant_load(f.read())
                    loaded = True
                except api.PkError as e:
                    return dict(status="load_fail", detail=str(e)[:300])
            try:
                fam, knobs, _ = self.ctx.variant_info(vid)
                if fam != api.FAMILY_IDS[self.family]:
                    return dict(status="load_fail", detail=f"family {fam}")
                res = dict(status="ok", knobs=knobs[:13])
                if req.get("validate", True):
                    seeds = list(range(int(req.get("seeds", 1))))
                    worst, where = self.validate(vid, seeds)
                    res["err"] = worst
                    if worst > 1.0:
                        res.update(status="wrong_output", detail=where)
                        return res
                if req.get("time", True):
                    sizes = [int(s) for s in req.get("sizes", [])]
                    try:
                        res["times"] = self.time(vid, sizes, int(req.get("replays", 1)), req.get("cutoff"))
                    except Implausible as e:
                        res.update(status="wrong_output", detail=str(e)[:300])
                return res
            finally:
                if loaded:
                    self.ctx.variant_unload(vid)
        raise ValueError(f"unknown op {op}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", required=True)
    ap.add_argument("--sizes", default=",".join(map(str, W.SIZES)))
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args()
    out = sys.stdout
    sys.stdout = sys.stderr      # nothing but protocol lines on the real stdout
    w = Worker(a.family, [int(s) for s in a.sizes.split(",")], a.reps)
    out.write(json.dumps({"ready": True, "family": a.family, "instances": [i.name for i in w.insts]}) + "\n")
    out.flush()
    for line in sys.stdin:
        line = line.strip()
        if not line:
            continue
        req = json.loads(line)
        if req.get("op") == "quit":
            break
        try:
            res = w.handle(req)
        except Exception as e:     # noqa: BLE001 - reported to the explorer, never fatal here
            res = dict(status="error", detail=f"{type(e).__name__}: {e}"[:500],
                       trace=traceback.format_exc()[-800:])
        res["id"] = req.get("id")
        out.write(json.dumps(res) + "\n")
        out.flush()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
