"""Benchmark of the mixed-size autotuned batch on one MI355X.

One step = one replay of the captured graph that runs every FP32 operation of
the library at N in {256, 512, 1000, 2048, 4096} plus the 3x3x3 stencil on a
256^3 volume, each with the variant the tuning table selects for its size.

Reported metric (one JSON line): the geometric mean, over all (operation,
size) instances, of default-variant time / tuned-variant time.  Each
instance is timed with HIP events as captured graphs of `--reps` and
2*`--reps` back-to-back launches on rotating operand copies (so the large
memory-bound instances read from HBM rather than from the 256 MB Infinity
Cache); the difference over `--reps` is its time per launch, free of the
graph launch cost.  The line also carries the reuse speedups (K = 1, 3),
the roofline position of the dominant kernel, every instance's GB/s or
GFLOP/s as a fraction of its roofline and of the measured device-copy
ceiling, the reduced-precision and next-row workloads, and the FP64 CPU
oracle timed on a bounded sample of the same batch.

    python bench.py [--steps K] [--warmup W] [--reps R] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_FP32 = 157.3e12       # flop/s, MI355X FP32 (matrix and vector)
PEAK_BF16 = 2516.6e12      # flop/s, MI355X dense BF16 MFMA
ROTATE_BYTES = 640 << 20   # per-instance graphs cycle through this much operand memory


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--reps", type=int, default=20, help="launches per per-instance timing graph")
    p.add_argument("--repeats", type=int, default=5, help="timed replays per per-instance graph")
    p.add_argument("--table", default=None, help="tuning table (default: the package's)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--sizes", default=None, help="comma-separated subset of sizes (testing)")
    p.add_argument("--profile", default=None, metavar="INSTANCE",
                   help="run only INSTANCE (e.g. gemm/4096) eagerly --steps times, for counter collection")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run a plain 256 MiB device copy --steps times (HBM counter calibration)")
    return p.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pk_gemm_4096_traffic.md")


def committed_traffic(code_hash: int):
    """HBM bytes per launch of the dominant kernel from the committed counter summary,
    or None when that summary was taken on a different code object."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 2:
                vals[cells[0]] = cells[1]
    try:
        if int(vals["code_hash"], 16) != code_hash:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy(steps):
    """A plain copy of known size for scaling the HBM byte counters."""
    import torch
    n = (256 << 20) // 4
    src = torch.rand(n, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": n * 4, "bytes_written": n * 4,
                      "launches": steps}), flush=True)


def profile_instance(names, steps, table):
    """Instances run one after another, eagerly, with the tuned variants: a clean
    dispatch stream for counters.  Prints each one's variant code hashes."""
    import torch
    from paper_1810_10496_amd import api, tuned, workloads as W
    ctx = api.context(0)
    applied = tuned.apply(ctx, table or tuned.TABLE)
    stream = torch.cuda.current_stream()
    for name in names.split(","):
        size = int(name.split("/")[1])
        pool = W.batch_instances((size,)) + W.precision_instances((size,)) + W.config_instances() + \
            W.corr_precision_instances((size,)) + W.next_instances()
        insts = [i for i in pool if i.name == name]
        if not insts:
            raise SystemExit(f"no instance {name}")
        inst = insts[0]
        inst.state = inst.make(torch.device("cuda:0"), 1)
        torch.cuda.synchronize()
        for _ in range(steps):
            inst.run(ctx, inst.state, 0, stream)
        torch.cuda.synchronize()
        hashes = {}
        for fam in inst.families:
            bucket = api.Context.size_bucket(size)
            vid = next((e["vid"] for e in applied if e["family"] == fam and int(e["bucket"]) == bucket
                        and e["vid"] >= 0), ctx.variant_default(fam))
            hashes[fam] = f"{ctx.variant_info(vid)[2]:016x}"
        print(json.dumps({"instance": name, "launches": steps, "algorithmic_bytes": inst.bytes,
                          "algorithmic_flops": inst.flops, "code_hash": hashes}), flush=True)
        inst.state = None
        torch.cuda.empty_cache()


def gpu_state():
    """Clock, power and performance-level readings of the GPU from rocm-smi (recorded next to
    the timing, as the timing protocol asks; the clocks a kernel actually ran at come from
    GRBM_GUI_ACTIVE, see the profiles)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--showpower", "--showperflevel", "--json"],
                           capture_output=True, text=True, timeout=30)
        doc = json.loads(r.stdout)
    except Exception as e:      # noqa: BLE001 -- informational only
        return {"error": f"{type(e).__name__}: {e}"[:200]}
    keep = ("clk", "power", "performance level")
    return {card: {k: v for k, v in vals.items() if any(t in k.lower() for t in keep)}
            for card, vals in doc.items() if isinstance(vals, dict)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The FP64 oracle timed per kernel at the measured workloads' sizes, with all of the
    host's threads and with one (operand generation outside the timing; median of 3 for
    calls under 1 s).  Single-threaded, the chained product and the correlation run at
    1024 instead of 2048 (about 20 s each otherwise); their rate is what is reported."""
    from oracle import oracle
    from paper_1810_10496_amd import synth

    def k_gemm(n):
        A, B, C, a, b = synth.gemm_inputs(n, workload=1)
        return (lambda: oracle.gemm(A, B, C, a, b)), 2.0 * n ** 3 + 3.0 * n * n, 16.0 * n * n

    def k_gemm3(n):
        A, B, C, D, a, b = synth.gemm3_inputs(n, workload=3)
        return (lambda: oracle.gemm3(A, B, C, D, a, b)), 4.0 * n ** 3 + 3.0 * n * n, 20.0 * n * n

    def k_pair(n):
        A, x, z = synth.gemv_inputs(n, workload=2)
        return (lambda: (oracle.gemv(A, x), oracle.gemv_t(A, z))), 4.0 * n * n, 4.0 * (n * n + 4 * n)

    def k_conv2d(n):
        g, taps = synth.conv2d_inputs(n, workload=2)
        return (lambda: oracle.conv2d(g, taps)), 17.0 * (n - 2) ** 2, 8.0 * n * n

    def k_conv3d(n):
        v, taps = synth.conv3d_inputs(n, workload=5)
        return (lambda: oracle.conv3d(v, taps)), 53.0 * (n - 2) ** 3, 8.0 * n ** 3

    def k_colstats(n):
        X, eps = synth.corr_inputs(n, workload=4)
        return (lambda: oracle.colstats(X, eps)), 4.0 * n * n, 4.0 * (n * n + 2 * n)

    def k_corr(n):
        X, eps = synth.corr_inputs(n, workload=4)
        return (lambda: oracle.corr(X, eps)), 4.0 * n * n + n * (n + 1) * n, 4.0 * (2 * n * n + 2 * n)

    plan = [("gemm", k_gemm, 512, 512), ("gemv_pair", k_pair, 4096, 4096), ("conv2d", k_conv2d, 4096, 4096),
            ("gemm3", k_gemm3, 2048, 1024), ("colstats", k_colstats, 4096, 4096), ("corr", k_corr, 2048, 1024),
            ("conv3d", k_conv3d, 256, 256)]

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
        if dt >= 1.0:
            return dt
        ts = [dt]
        for _ in range(2):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    all_threads = oracle.num_threads()
    rows, flops_all, secs_all = [], 0.0, 0.0
    try:
        for name, make, n_all, n_one in plan:
            fn, fl, by = make(n_all)
            oracle.set_threads(all_threads)
            t_all = timed(fn)
            if n_one != n_all:
                fn, fl1, by1 = make(n_one)
            else:
                fl1, by1 = fl, by
            oracle.set_threads(1)
            t_one = timed(fn)
            del fn
            flops_all += fl
            secs_all += t_all
            rows.append(dict(kernel=name, size=n_all, all_threads_s=round(t_all, 4),
                             all_threads_gflops=round(fl / t_all / 1e9, 2), all_threads_gbs=round(by / t_all / 1e9, 2),
                             one_thread_size=n_one, one_thread_s=round(t_one, 4),
                             one_thread_gflops=round(fl1 / t_one / 1e9, 3)))
    finally:
        oracle.set_threads(all_threads)
    return dict(value=round(flops_all / secs_all / 1e9, 3), unit="GFLOP/s (algorithmic, FP64 oracle, all threads)",
                cores=all_threads, kind="oracle", cpu=_cpu_model(),
                sample="one call of each kernel at its workload size (gemm 512, matvec pair 4096^2, 2D stencil "
                       "4096^2, chained product 2048, column statistics 4096^2, correlation 2048, 3D stencil "
                       "256^3); one thread: chained product and correlation at 1024",
                seconds=round(secs_all, 3), per_kernel=rows)


# read-dominated operations are measured against the read ceiling, the stencils (one
# read and one write of the grid) against the copy ceiling
READ_OPS = ("gemv", "gemv_t", "gemv_pair", "colstats", "gesummv", "mvt")


def ceiling_for(op, read_gbs, copy_gbs):
    return ("read", read_gbs) if op in READ_OPS else ("copy", copy_gbs)


def stream_ceilings(ctx, dev, stream, rounds=8):
    """GB/s of the library's read and copy probes over four 512 MiB buffers in turn."""
    import torch
    n = (512 << 20) // 4
    bufs = [torch.rand(n, device=dev) for _ in range(4)]
    sums = torch.empty(ctx.STREAM_BLOCKS, device=dev)
    dsts = [torch.empty(n, device=dev) for _ in range(2)]
    torch.cuda.synchronize()
    out = {}
    for kind in ("read", "read_nt", "copy", "copy_nt"):
        def one(r):
            if kind.startswith("read"):
                ctx.stream_probe(kind, bufs[r % 4], sums, stream=stream)
            else:
                ctx.stream_probe(kind, bufs[r % 4], dsts[r % 2], stream=stream)
        for r in range(4):
            one(r)
        ctx.timer_start(stream)
        for r in range(4 * rounds):
            one(r)
        ms = ctx.timer_stop(stream)
        moved = n * 4 * (1 if kind.startswith("read") else 2) * 4 * rounds
        out[kind] = moved / (ms * 1e-3) / 1e9
    # torch's own device copy, for reference
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        dsts[0].copy_(bufs[0])
        e0.record(stream)
        for r in range(4 * rounds):
            dsts[r % 2].copy_(bufs[r % 4])
        e1.record(stream)
    e1.synchronize()
    out["torch_copy"] = n * 4 * 2 * 4 * rounds / (e0.elapsed_time(e1) * 1e-3) / 1e9
    # the ceilings: the faster form of each probe
    out["read_ceiling"] = max(out["read"], out["read_nt"])
    out["copy_ceiling"] = max(out["copy"], out["copy_nt"], out["torch_copy"])
    del bufs, dsts
    torch.cuda.empty_cache()
    return out


def vendor_blas(dev):
    """The vendor BLAS (torch.matmul on ROCm: hipBLASLt) at the dense products' sizes, as
    context for the roofline fractions: FP32 (no reduced-precision shortcut) and BF16,
    square 2048 and 4096, per-call time from a graph of 20 calls, median of 5 replays."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    out = []
    for dt, name, peak in ((torch.float32, "fp32", PEAK_FP32), (torch.bfloat16, "bf16", PEAK_BF16)):
        for n in (2048, 4096):
            A = torch.rand(n, n, device=dev).to(dt)
            B = torch.rand(n, n, device=dev).to(dt)
            C = torch.empty(n, n, device=dev, dtype=dt)
            for _ in range(3):
                torch.matmul(A, B, out=C)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                for _ in range(20):
                    torch.matmul(A, B, out=C)
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                g.replay()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) / 20)
            t = statistics.median(ts)
            tf = 2.0 * n ** 3 / (t * 1e-3) / 1e12
            out.append(dict(dtype=name, n=n, us=round(t * 1e3, 1), tflops=round(tf, 1), frac=round(tf * 1e12 / peak, 4)))
            del g, A, B, C
            torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}); the kernels run on one "
              "GPU's share of the work, and no multi-GPU path is measured", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy(args.steps)
        return
    if args.profile:
        profile_instance(args.profile, args.steps, args.table)
        return

    import torch
    from paper_1810_10496_amd import api, tuned, workloads as W
    from paper_1810_10496_amd.timing import per_launch_ms

    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    ctx = api.context(0)
    stream = torch.cuda.Stream()

    sizes = tuple(int(s) for s in args.sizes.split(",")) if args.sizes else W.SIZES
    insts = W.batch_instances(sizes)
    log(f"{len(insts)} instances; allocating operands")
    for inst in insts:
        copies = 1
        if inst.footprint > 0:
            copies = max(1, min(args.reps, math.ceil(ROTATE_BYTES / inst.footprint)))
        inst.state = inst.make(dev, copies)
        inst.state["_copies"] = copies
    torch.cuda.synchronize()

    applied = tuned.apply(ctx, args.table or tuned.TABLE)
    chosen = {}   # (family, bucket) -> vid
    for e in applied:
        if e["vid"] >= 0:
            chosen[(e["family"], int(e["bucket"]))] = e["vid"]
    log(f"tuning table: {len(applied)} entries, {sum(1 for e in applied if e['vid'] >= 0)} usable")

    reuse = tuned.load_reuse(ctx, args.table or tuned.TABLE)
    sides = ["default", "tuned"] + (["k1", "k3"] if reuse else [])
    log(f"reuse assignments: {len(reuse)}")

    def variant_kind(inst):
        ents = [e for e in applied if e["family"] in inst.families
                and int(e["bucket"]) == api.Context.size_bucket(inst.size) and e["vid"] >= 0
                and not e.get("is_default")]
        if not ents:
            return "default kept"
        from paper_1810_10496_amd import codegen
        knobs = any(dict(e["knobs"]) != dict(codegen.FAMILIES[e["family"]].defaults) for e in ents)
        pipe = any(e["pipeline"] != codegen.DEFAULT_PIPELINE or e.get("opt_flags")
                   or list(e.get("llc_flags", ["-O3"])) != ["-O3"] for e in ents)
        return {(True, False): "knobs only", (False, True): "pipeline only"}.get((knobs, pipe), "knobs and pipeline")

    def variant_for(fam, size, side):
        if side == "tuned":
            vid = chosen.get((fam, api.Context.size_bucket(size)))
            if vid is not None:
                return vid
        elif side in ("k1", "k3"):
            vid = reuse.get((fam, size, int(side[1])))
            if vid is not None:
                return vid
        return ctx.variant_default(fam)

    def side_time(inst, side, replays):
        """ms per launch of `inst` with the `side` variants (graph launch cost excluded)."""
        for fam in inst.families:
            ctx.variant_select(fam, variant_for(fam, inst.size, side))
        try:
            return per_launch_ms(ctx, stream, lambda i: inst.run(ctx, inst.state, i % inst.state["_copies"], stream),
                                 args.reps, replays)
        finally:
            for fam in inst.families:
                ctx.variant_select(fam, -1)
    # the batch: every instance once, tuned variants through the table
    with ctx.capture(stream) as batch:
        for inst in insts:
            inst.run(ctx, inst.state, 0, stream)

    for _ in range(args.warmup):
        batch.launch(stream)
    stream.synchronize()

    state = gpu_state()
    # ---- timed region: K steps of the batch ------------------------------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.timer_start(stream)
    for _ in range(args.steps):
        batch.launch(stream)
    ev_ms = ctx.timer_stop(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ms_per_step = ev_ms / args.steps

    # ---- the chip's practical HBM ceilings, from the library's own probes: every element
    # of a buffer read once, and a copy; 512 MiB buffers in turn (2 GiB read, 1 GiB copied
    # per round), far beyond the 256 MB Infinity Cache
    ceil = stream_ceilings(ctx, dev, stream)
    read_gbs, copy_gbs = ceil["read_ceiling"], ceil["copy_ceiling"]
    log(f"HBM ceilings: read {read_gbs:.0f} GB/s, copy {copy_gbs:.0f} GB/s")

    # ---- per-instance default vs tuned ----------------------------------------------------------
    rows = []
    for inst in insts:
        ts = {side: [] for side in sides}
        for _ in range(args.repeats):          # sides interleaved, so drift hits them alike
            for side in sides:
                ts[side].append(side_time(inst, side, 1))
        med = {side: statistics.median(v) for side, v in ts.items()}
        tdm, ttm = med["default"], med["tuned"]
        if inst.bound == "hbm":
            ach, peak, unit = inst.bytes / (ttm * 1e-3), PEAK_HBM, "GB/s"
        else:
            ach, peak, unit = inst.flops / (ttm * 1e-3), PEAK_FP32, "GFLOP/s"
        rows.append(dict(instance=inst.name, default_us=round(tdm * 1e3, 2), tuned_us=round(ttm * 1e3, 2),
                         speedup=round(tdm / ttm, 4), achieved=round(ach / 1e9, 1), unit=unit,
                         frac=round(ach / peak, 4), gflops=round(inst.flops / (ttm * 1e-3) / 1e9, 1)))
        if inst.bound == "hbm":
            kind, cg = ceiling_for(inst.op, read_gbs, copy_gbs)
            rows[-1]["frac_of_ceiling"] = round(ach / 1e9 / cg, 4)
            rows[-1]["ceiling"] = kind
        rows[-1]["variant"] = variant_kind(inst)
        for side in ("k1", "k3"):
            if side in med:
                rows[-1][f"reuse_{side}_us"] = round(med[side] * 1e3, 2)
                rows[-1][f"reuse_{side}_speedup"] = round(tdm / med[side], 4)

    def gm(key, sel=None):
        vals = [r[key] for r in rows if sel is None or sel(r)]
        return round(math.exp(sum(math.log(v) for v in vals) / len(vals)), 4) if vals else None
    geo = gm("speedup")
    by_size = {str(z): gm("speedup", lambda r, z=z: r["instance"].endswith(f"/{z}")) for z in sizes}
    by_size[str(W.CONV3D_SIZE) + "^3"] = gm("speedup", lambda r: r["instance"].startswith("conv3d/"))
    # where the tuned speedups come from: instances whose tuned variants differ from the
    # default only in knobs (standard -O3 pipeline), those whose pipeline changed too, and
    # those that kept the built-in default
    split = {k: dict(instances=sum(1 for r in rows if r["variant"] == k), geomean=gm("speedup", lambda r, k=k:
                                                                                      r["variant"] == k))
             for k in ("knobs only", "pipeline only", "knobs and pipeline", "default kept")}

    # dominant kernel: pk_gemm at the largest GEMM instance, tuned variant
    big = max((r for r in rows if r["instance"].startswith("gemm/")), key=lambda r: int(r["instance"].split("/")[1]))
    n = int(big["instance"].split("/")[1])
    big_bytes = next(i.bytes for i in insts if i.name == big["instance"])
    gflop = (2.0 * n ** 3 + 3.0 * n * n) / 1e9
    t_s = big["tuned_us"] * 1e-6
    gemm_vid = variant_for("gemm_f32", n, "tuned")
    code_hash = ctx.variant_info(gemm_vid)[2]
    roof = dict(kernel="pk_gemm", instance=big["instance"] + " fp32 tuned", bound="mfma",
                achieved=round(gflop / t_s / 1e3, 2), peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                frac=round(gflop / t_s / 1e3 / (PEAK_FP32 / 1e12), 4), traffic=committed_traffic(code_hash),
                traffic_unit="bytes per launch (HBM, counter-derived)", code_hash=f"{code_hash:016x}",
                algorithmic_bytes_per_launch=big_bytes,
                avg_launch_us=big["tuned_us"], algorithmic_gflop_per_launch=round(gflop, 3))

    # ---- workloads outside the batch: the contractions in FP32, BF16 and split BF16, and
    # the next rows (COVAR, SYRK, SYR2K, GESUMMV, MVT, FDTD-2D); tuned variants where tuned
    def time_outside(extra, with_default=False):
        out_rows = []
        for inst in extra:
            copies = max(1, min(args.reps, math.ceil(ROTATE_BYTES / max(inst.footprint, 1))))
            inst.state = inst.make(dev, copies)
            inst.state["_copies"] = copies
            t = side_time(inst, "tuned", args.repeats)
            td = side_time(inst, "default", args.repeats) if with_default else None
            inst.state = None
            torch.cuda.empty_cache()
            row = dict(instance=inst.name, us=round(t * 1e3, 2))
            if td is not None:
                row.update(default_us=round(td * 1e3, 2), speedup=round(td / t, 4))
            if inst.bound == "hbm":
                gbs = inst.bytes / (t * 1e-3) / 1e9
                kind, cg = ceiling_for(inst.op, read_gbs, copy_gbs)
                row.update(gbs=round(gbs, 1), peak_gbs=PEAK_HBM / 1e9, frac=round(gbs * 1e9 / PEAK_HBM, 4),
                           frac_of_ceiling=round(gbs / cg, 4), ceiling=kind)
            elif inst.bound == "infinity_cache":
                # the operands stay in the 256 MB Infinity Cache across the call: no HBM figure
                row.update(gbs=round(inst.bytes / (t * 1e-3) / 1e9, 1), bound="infinity_cache")
            else:
                tf = inst.flops / (t * 1e-3) / 1e12
                fam = inst.families[-1]
                low = "bf16" in fam or "split" in fam
                peak = PEAK_BF16 / 1e12 if low else PEAK_FP32 / 1e12
                row.update(tflops=round(tf, 2), peak_tflops=peak, frac=round(tf / peak, 4))
                if "split" in fam:
                    row["mfma_frac"] = round(3 * tf / peak, 4)    # three bf16 products per useful one
            out_rows.append(row)
        return out_rows

    # ---- the phase-order exploration's best orders (default knobs, random pass orders,
    # minimised) against the default pipeline, each at its family's benchmark size
    order_rows = []
    if not args.sizes:
        for fam, (vid, e) in sorted(tuned.load_orders(ctx).items()):
            for inst in W.family_instances(fam, (e["size"],)):
                copies = max(1, min(args.reps, math.ceil(ROTATE_BYTES / max(inst.footprint, 1))))
                inst.state = inst.make(dev, copies)
                inst.state["_copies"] = copies
                ts = {"default": [], "order": []}
                for _ in range(args.repeats):
                    for side, v in (("default", ctx.variant_default(fam)), ("order", vid)):
                        ctx.variant_select(fam, v)
                        try:
                            ts[side].append(per_launch_ms(ctx, stream, lambda i: inst.run(
                                ctx, inst.state, i % inst.state["_copies"], stream), args.reps, 1))
                        finally:
                            ctx.variant_select(fam, -1)
                td, to = statistics.median(ts["default"]), statistics.median(ts["order"])
                order_rows.append(dict(family=fam, instance=inst.name, default_us=round(td * 1e3, 2),
                                       order_us=round(to * 1e3, 2), speedup=round(td / to, 4),
                                       passes=len(e["pipeline"].split(","))))
                inst.state = None
                torch.cuda.empty_cache()
        if order_rows:
            log(f"phase orders: {len(order_rows)} families timed")

    prec_rows, next_rows = [], []
    if not args.sizes:
        prec_rows = time_outside(W.config_instances() + W.precision_instances((4096,)))
        next_rows = time_outside(W.next_instances(), with_default=True)
        log(f"outside the batch: {len(prec_rows)} precision and {len(next_rows)} next-row workloads timed")

    step_flops = sum(i.flops for i in insts)
    out = {
        "metric": "geomean tuned-vs-default speedup; GFLOP/s, GB/s as % of roofline",
        "value": round(geo, 4),
        "unit": "x (geomean over batch instances)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "wall_ms_per_step": round(wall_ms / args.steps, 4),
        "step_gflops": round(step_flops / (ms_per_step * 1e-3) / 1e9, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded SplitMix64: uniform [0,1) operands, normal+offset correlation data)",
        "config": {"workload": "mixed-size autotuned batch: gemm, gemm3, gemv, gemv_t, gemv_pair, conv2d, "
                               "colstats, corr at N in " + ",".join(map(str, sizes)) + "; conv3d 256^3",
                   "instances": len(insts), "tuned_entries": len(chosen), "reps_per_timing_graph": args.reps},
        "roofline": roof,
        "hbm_ceilings_gbs": {k: round(v, 1) for k, v in ceil.items()},
        "geomean_by_size": by_size,
        "speedup_sources": split,
        "reuse": ({"cosine_k1": round(gm("reuse_k1_speedup"), 4), "cosine_k3": round(gm("reuse_k3_speedup"), 4),
                   "tuner_estimates": tuned.reuse_summary(args.table or tuned.TABLE)} if reuse else None),
        "phase_orders": ({"geomean": round(math.exp(sum(math.log(r["speedup"]) for r in order_rows)
                                                   / len(order_rows)), 4), "rows": order_rows}
                         if order_rows else None),
        "instances": rows,
        "precisions": prec_rows,
        "next_rows": next_rows,
        "gpu_state_before_timing": state,
    }
    log("timing the vendor BLAS (torch.matmul) at the dense products' sizes, for context")
    out["vendor_blas"] = vendor_blas(dev)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline()
    batch.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
