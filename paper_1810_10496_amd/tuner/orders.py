"""The phase-order exploration: the paper's own experiment (Sec. 3) on these kernels.

The kernel source is fixed (each family at its default knobs) and only the LLVM
pass sequence applied to its un-optimised device IR varies, as in the paper's
compilation flow (Sec. 2.3): front end -> `opt` with the order -> AMDGPU `llc`
-> `lld`.  Experiments, all on one seeded set of orders shared by every family
(Sec. 3 opening):

  sample    N random orders of 1..256 pool passes, drawn uniformly with
            repetition (the pool: `tuner.passes`); each compiled on the host,
            every code object through the gate (`tuner.gate`), then each
            distinct code object validated and timed once on the GPU at the
            family's benchmark size (Sec. 2.1, 2.4).  The evaluation stops at
            the first worker that dies or hangs: such a candidate may have
            faulted the GPU, and nothing more runs on it after that.
  census    outcome classes over the sample (Sec. 3.2): no optimised IR
            (`no_output`), back-end failure (`compile_fail`), held back by the
            gate (`gated`), wrong output, time-out, crash, broken report, ok.
  finalize  the ten fastest re-timed with 30 replays, the fastest validated
            with 30 seeds (Sec. 2.1, 2.4), against the built-in default
            (`default<O3>`); the best order is kept for the later experiments
            whether or not it beats the default, and its speedup is reported.
  minimise  Table 1: pass instances that change nothing are removed -- first
            those whose removal leaves the code object's bytes unchanged
            (host only), then those whose removal does not slow the kernel by
            more than `MARGIN` (timed on the GPU, the order compiled there).
  permute   up to 1000 distinct random permutations of each minimised order
            (the same pass instances, Sec. 3.3), timed relative to it.
  cross     each family's minimised order applied to every other family,
            relative to that family's own (Sec. 3.3, the sequence matrix).
  first100 / convergence: from the sample's single timings (Sec. 3.3).

    python -m paper_1810_10496_amd.tuner orders-build   --workdir W --samples 1000
    python -m paper_1810_10496_amd.tuner orders-eval    --workdir W --codir C    (GPU)
    python -m paper_1810_10496_amd.tuner orders-finalize --workdir W             (GPU)
    python -m paper_1810_10496_amd.tuner orders-minimise --workdir W [--stage host|gpu]
    python -m paper_1810_10496_amd.tuner orders-permute  --workdir W [--stage host|gpu]
    python -m paper_1810_10496_amd.tuner orders-cross    --workdir W [--stage host|gpu]
    python -m paper_1810_10496_amd.tuner orders-report   --workdir W --out orders.md
"""
from __future__ import annotations

import concurrent.futures as cf
import itertools
import json
import math
import os
import random
import statistics

from .. import codegen, workloads as W
from . import explore as X, gate, space
from .evaluator import Evaluator

# the FP32 families of the paper's kernels: GEMM and 2MM/3MM, ATAX/BICG/MVT (matvec,
# transposed, fused pair), 2DCONV, 3DCONV, CORR (column statistics, rank-k), SYRK/SYR2K,
# GESUMMV, FDTD-2D
FAMILIES = ("gemm_f32", "gemv", "gemv_t", "gemv_pair", "conv2d", "conv3d", "colstats", "syrk_f32",
            "rankk", "gesummv", "fdtd")
ORDER_SEED = 5501
MAX_LEN = 256
MARGIN = 0.02           # a pass stays in a minimised order if removing it costs more than this
PERMUTATIONS = 1000


def family_size(family: str) -> int:
    """The size each family is explored at: its largest benchmark instance."""
    return W.CONV3D_SIZE if family == "conv3d" else max(W.SIZES)


def sample_orders(pool: list[str], count: int, seed: int = ORDER_SEED, max_len: int = MAX_LEN) -> list[list[str]]:
    """`count` orders, each 1..max_len pool entries drawn uniformly with repetition."""
    rng = random.Random(f"{seed}:orders")
    return [[rng.choice(pool) for _ in range(rng.randint(1, max_len))] for _ in range(count)]


def pipeline(order: list[str]) -> str:
    return ",".join(order)


def order_variant(family: str, order: list[str]) -> space.Variant:
    return space.Variant(family, space.default_knobs(family), pipeline(order))


def sample_variants(family: str, orders: list[list[str]]) -> list[space.Variant]:
    return [order_variant(family, o) for o in orders]


def _load(workdir, name, default=None):
    p = os.path.join(workdir, name)
    if not os.path.exists(p):
        return default
    with open(p) as f:
        return json.load(f)


def _save(workdir, name, doc):
    os.makedirs(workdir, exist_ok=True)
    p = os.path.join(workdir, name)
    with open(p + ".tmp", "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    os.replace(p + ".tmp", p)


def load_orders(workdir) -> list[list[str]]:
    doc = _load(workdir, "orders.json")
    if doc is None:
        raise FileNotFoundError(f"{workdir}/orders.json: run orders-build first")
    return doc["orders"]


# ------------------------------------------------------------------------ sample --

def build(families, workdir, pool, count, seed=ORDER_SEED, jobs=8, log=print):
    """Host side of the sample: draw the orders, compile every (family, order)."""
    orders = sample_orders(pool, count, seed)
    _save(workdir, "orders.json", dict(seed=seed, max_len=MAX_LEN, count=count, pool=pool, orders=orders))
    db = X.DB(os.path.join(workdir, "db.jsonl"))
    out = {}
    for fam in families:
        vs = [space.default_variant(fam)] + sample_variants(fam, orders)
        recs = X._build_many(db, vs, workdir, jobs)
        c = {}
        for r in recs[1:]:
            c[r["status"]] = c.get(r["status"], 0) + 1
        c["distinct_code_objects"] = len({r["sha"] for r in recs[1:] if r["status"] == "ok"})
        out[fam] = c
        log(f"[orders] {fam}: built {count} orders: {json.dumps(c, sort_keys=True)}")
    return out


def evaluate(families, workdir, jobs=8, log=print, eval_timeout=120.0, max_minutes=None):
    """GPU side of the sample: validate and time every distinct code object once
    (resumable: a later call continues where a time limit stopped this one)."""
    import time
    orders = load_orders(workdir)
    res = {}
    t0 = time.time()
    for fam in families:
        left = None if max_minutes is None else max_minutes - (time.time() - t0) / 60.0
        if left is not None and left <= 0:
            log(f"[orders] time limit reached before {fam} (resumable)")
            break
        vs = [space.default_variant(fam)] + sample_variants(fam, orders)
        res[fam] = X.explore(fam, workdir, sizes=(family_size(fam),), jobs=jobs, log=log, variants=vs,
                             eval_timeout=eval_timeout, stop_on_failure=True, max_minutes=left)
        log(f"[orders] {fam} census: {json.dumps(res[fam], sort_keys=True)}")
    return res


def census(workdir, families):
    """Outcome counts per family over the sample; compile failures are split by stage
    into `no_ir` (opt crashed or produced nothing: the paper's "optimised IR not
    generated") and `backend_fail` (llc or lld rejected the optimised IR)."""
    db = X.DB(os.path.join(workdir, "db.jsonl"))
    orders = load_orders(workdir)
    out = {}
    for f in families:
        keys = {v.key() for v in sample_variants(f, orders)}
        c = X.census(db, f, keys)
        latest = {}
        for r in db.where(kind="compile", family=f):
            if r["key"] in keys:
                latest[r["key"]] = r
        fails = [r for r in latest.values() if r["status"] == "compile_fail"]
        c.pop("compile_fail", None)
        c["no_ir"] = c.pop("no_output", 0) + sum(1 for r in fails if r.get("stage") in ("opt", "frontend"))
        c["backend_fail"] = sum(1 for r in fails if r.get("stage") not in ("opt", "frontend"))
        out[f] = c
    return out


def finalize(families, workdir, log=print):
    """Per family, the best sampled order at its size (30 replays, 30-seed validation) and
    the default's time; the order is kept even when it does not beat the default (an
    order that builds the default's own code object does not count as found)."""
    doc = _load(workdir, "best.json", {})
    db = X.DB(os.path.join(workdir, "db.jsonl"))
    for fam in families:
        size = family_size(fam)
        # the sampled random orders compete, not the default pipeline's own code object
        dkey = space.default_variant(fam).key()
        own = {r["sha"] for r in db.where(kind="compile", family=fam, status="ok") if r["key"] == dkey}
        ents = X.finalize(fam, workdir, sizes=(size,), log=log, margin=-1.0, exclude=own)
        e = ents[0]
        if e.get("is_default"):
            doc[fam] = dict(size=size, order=None, default_ms=e["default_ms"])
        else:
            doc[fam] = dict(size=size, order=e["pipeline"].split(","), default_ms=e["default_ms"],
                            best_ms=e["tuned_ms"], speedup=e["speedup"], code_sha256=e["code_sha256"])
        _save(workdir, "best.json", doc)
        log(f"[orders] {fam}: best order {doc[fam].get('speedup', float('nan')):.3f}x the default")
    return doc


# ---------------------------------------------------------------------- minimise --

def _hash(family, order):
    try:
        b = codegen.compile_variant(family, space.default_knobs(family), pipeline(order), timeout=180)
    except codegen.CompileError:
        return None
    return b.code_hash


def strip_inert(family, order, jobs=8, log=print):
    """Remove pass instances whose removal leaves the code object's bytes unchanged.

    Chunks of halving size are tried at each granularity: the removals of one
    granularity are tested in parallel against the current order, applied all at
    once if together they still leave the bytes unchanged, else one at a time."""
    ref = _hash(family, order)
    if ref is None:
        raise RuntimeError(f"{family}: the order to minimise does not build")
    cur = list(order)
    chunk = max(1, len(cur) // 2)
    compiles = 1
    while True:
        spans = [(i, min(i + chunk, len(cur))) for i in range(0, len(cur), chunk)]
        cands = [cur[:a] + cur[b:] for a, b in spans]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            hs = list(ex.map(lambda o: _hash(family, o) if o else None, cands))
        compiles += len(cands)
        inert = [sp for sp, h in zip(spans, hs) if h == ref]
        if inert:
            drop = set()
            for a, b in inert:
                drop.update(range(a, b))
            together = [p for i, p in enumerate(cur) if i not in drop]
            compiles += 1
            if together and _hash(family, together) == ref:
                cur = together
            else:
                for a, b in reversed(inert):       # right to left keeps earlier indices valid
                    trial = cur[:a] + cur[b:]
                    compiles += 1
                    if trial and _hash(family, trial) == ref:
                        cur = trial
        if chunk == 1:
            break
        chunk = max(1, chunk // 2)
    log(f"[orders] {family}: {len(order)} -> {len(cur)} passes with identical code ({compiles} compiles)")
    return cur, ref


def minimise_host(families, workdir, jobs=8, log=print):
    best = _load(workdir, "best.json", {})
    doc = _load(workdir, "minimised.json", {})
    for fam in families:
        b = best.get(fam)
        if not b or not b.get("order"):
            continue
        if fam in doc and doc[fam].get("from") == b["order"]:
            continue
        inert_free, sha = strip_inert(fam, b["order"], jobs, log)
        doc[fam] = dict(size=b["size"], **{"from": b["order"]}, same_code=inert_free, code_sha256=sha)
        _save(workdir, "minimised.json", doc)
    return doc


def minimise_gpu(families, workdir, replays=10, jobs=16, log=print, make_evaluator=None, build=None):
    """Remove the remaining passes whose removal does not slow the kernel by more than
    MARGIN.  Every single-pass removal is built (in parallel) and timed against the
    order itself; the passes whose removal alone stays within MARGIN are then removed
    together if that still stays within MARGIN, else one at a time, last to first, each
    judged against the order it starts from."""
    doc = _load(workdir, "minimised.json", {})
    db = X.DB(os.path.join(workdir, "db_minimise.jsonl"))

    build = build or X._build

    def timed(ev, fam, order, size, rec=None):
        rec = rec or build(order_variant(fam, order), workdir)
        db.add(rec)
        if rec["status"] != "ok":
            return rec["status"], None, None
        e = X._evaluate(ev, db, fam, rec["sha"], X._co_path(workdir, fam, rec["sha"]), [size], None, 300,
                        replays=replays, validate=True)
        if e["status"] in ("crashed", "timeout"):
            ev.close()
            raise X.WorkerFailure(f"{fam}: worker {e['status']}; stopping")
        return e["status"], (e["times"].get(str(size)) if e["status"] == "ok" else None), rec["sha"]

    for fam in families:
        m = doc.get(fam)
        if not m or "minimal" in m:
            continue
        size = m["size"]
        ev = (make_evaluator or (lambda f, z: Evaluator(f, [z], log=log, stderr_path=os.path.join(
            workdir, f"worker_{f}.err"))))(fam, size)
        st, t0, _ = timed(ev, fam, m["same_code"], size)
        if st != "ok" or not t0:
            ev.close()
            m["minimal"], m["note"] = m["same_code"], f"the order itself: {st}"
            _save(workdir, "minimised.json", doc)
            continue
        cur = list(m["same_code"])
        limit = t0 * (1.0 + MARGIN)
        trials = [cur[:i] + cur[i + 1:] for i in range(len(cur))]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            recs = list(ex.map(lambda o: build(order_variant(fam, o), workdir) if o else None, trials))
        singles = []
        for i, (o, rec) in enumerate(zip(trials, recs)):
            if rec is None:
                continue
            st, t, _ = timed(ev, fam, o, size, rec)
            singles.append(dict(removed=cur[i], position=i, status=st, ms=t,
                                removable=bool(st == "ok" and t and t <= limit)))
        drop = [x["position"] for x in singles if x["removable"]]
        together = [p for i, p in enumerate(cur) if i not in set(drop)]
        how = "none removable"
        if drop and together:
            st, t, _ = timed(ev, fam, together, size)
            if st == "ok" and t and t <= limit:
                cur, how = together, "removed together"
            else:
                how = "one at a time"
                for i in sorted(drop, reverse=True):
                    trial = cur[:i] + cur[i + 1:]
                    if not trial:
                        continue
                    st, t, _ = timed(ev, fam, trial, size)
                    if st == "ok" and t and t <= limit:
                        cur = trial
        st, t1, sha1 = timed(ev, fam, cur, size)
        d = X._evaluate(ev, db, fam, "default", "default", [size], None, 300, replays=replays, validate=False)
        ev.close()
        m.update(minimal=cur, singles=singles, how=how, ms_same_code=t0, ms_minimal=t1, status_minimal=st,
                 minimal_sha256=sha1, default_ms=d["times"].get(str(size)))
        _save(workdir, "minimised.json", doc)
        log(f"[orders] {fam}: minimal order {pipeline(cur)} ({t1} ms vs {t0} ms, {how})")
    return doc


# ----------------------------------------------------------------------- permute --

def permutations(order, count=PERMUTATIONS, seed=ORDER_SEED):
    """Up to `count` distinct orderings of the same pass instances (all of them when
    there are at most `count`), the order itself excluded."""
    base = tuple(order)
    distinct = set(itertools.permutations(base)) if len(base) <= 7 else None
    if distinct is not None:
        out = sorted(p for p in distinct if p != base)
        return [list(p) for p in out[:count]]
    rng = random.Random(f"{seed}:perm:{pipeline(order)}")
    seen, out = {base}, []
    tries = 0
    while len(out) < count and tries < 50 * count:
        tries += 1
        p = list(base)
        rng.shuffle(p)
        if tuple(p) not in seen:
            seen.add(tuple(p))
            out.append(p)
    return out


def _minimal(doc, fam):
    m = doc.get(fam) or {}
    return m.get("minimal") or m.get("same_code")


def permute_host(families, workdir, jobs=8, log=print):
    mins = _load(workdir, "minimised.json", {})
    db = X.DB(os.path.join(workdir, "db_permute.jsonl"))
    plan = _load(workdir, "permute_plan.json", {})
    for fam in families:
        order = _minimal(mins, fam)
        if not order:
            continue
        perms = permutations(order)
        vs = [order_variant(fam, order)] + [order_variant(fam, p) for p in perms]
        recs = X._build_many(db, vs, workdir, jobs)
        plan[fam] = dict(order=order, count=len(perms),
                         distinct=len({r["sha"] for r in recs if r["status"] == "ok"}))
        log(f"[orders] {fam}: {len(perms)} permutations, {plan[fam]['distinct']} distinct code objects")
    _save(workdir, "permute_plan.json", plan)
    return plan


class TimeLimit(RuntimeError):
    """The evaluation budget of a call ran out (resumable)."""


def _eval_set(fam, workdir, dbname, variants, size, replays, log, eval_timeout=120.0, deadline=None):
    """Validate and time every distinct built code object of `variants` once (with
    `replays` replays), stopping at the first worker that dies or hangs; TimeLimit when
    `deadline` (time.time()) passes first."""
    import time
    db = X.DB(os.path.join(workdir, dbname))
    keys = {v.key() for v in variants}
    recs = {}
    for r in db.where(kind="compile", family=fam):
        if r["key"] in keys:
            recs[r["key"]] = r
    shas = []
    for v in variants:
        r = recs.get(v.key())
        if r and r["status"] == "ok" and r["sha"] not in shas:
            shas.append(r["sha"])
    done = {r["sha"]: r for r in db.where(kind="eval", family=fam)}
    ev = Evaluator(fam, [size], log=log, stderr_path=os.path.join(workdir, f"worker_{fam}.err"))
    for sha in shas:
        if sha in done:
            continue
        p = X._co_path(workdir, fam, sha)
        if not os.path.exists(p):
            continue
        if deadline is not None and time.time() > deadline:
            ev.close()
            raise TimeLimit(f"{fam}: time limit reached (resumable)")
        e = X._evaluate(ev, db, fam, sha, p, [size], None, eval_timeout, replays=replays, validate=True)
        done[sha] = e
        t = e.get("times", {}).get(str(size))
        log(f"[orders] {fam} {dbname}: {len(done)}/{len(shas)} {e['status']} {sha[:10]} "
            f"{'%.4f ms' % t if t else ''}")
        if e["status"] in ("crashed", "timeout"):
            ev.close()
            raise RuntimeError(f"{fam}: worker {e['status']} on {sha[:12]}; stopping")
    ev.close()
    out = {}
    for v in variants:
        r = recs.get(v.key())
        if not r or r["status"] != "ok":
            out[v.pipeline] = (r or {}).get("status", "missing"), None
            continue
        e = done.get(r["sha"], {})
        out[v.pipeline] = e.get("status", "missing"), e.get("times", {}).get(str(size))
    return out


def permute_gpu(families, workdir, replays=3, log=print, max_minutes=None):
    import time
    plan = _load(workdir, "permute_plan.json", {})
    doc = _load(workdir, "permuted.json", {})
    deadline = None if max_minutes is None else time.time() + 60.0 * max_minutes
    for fam in families:
        if fam not in plan or fam in doc:
            continue
        order = plan[fam]["order"]
        size = family_size(fam)
        vs = [order_variant(fam, order)] + [order_variant(fam, p) for p in permutations(order)]
        try:
            res = _eval_set(fam, workdir, "db_permute.jsonl", vs, size, replays, log, deadline=deadline)
        except TimeLimit as e:
            log(f"[orders] {e}")
            return doc
        t0 = res[pipeline(order)][1]
        ratios, fails = [], {}
        for v in vs[1:]:
            st, t = res[v.pipeline]
            if st == "ok" and t and t0:
                ratios.append(t0 / t)
            else:
                fails[st] = fails.get(st, 0) + 1
        doc[fam] = dict(order=order, size=size, ms=t0, ratios=ratios, failures=fails)
        _save(workdir, "permuted.json", doc)
        log(f"[orders] {fam}: {len(ratios)} permutations timed, failures {fails}")
    return doc


# ------------------------------------------------------------------------- cross --

def cross_variants(families, mins):
    return {t: [(s, order_variant(t, _minimal(mins, s))) for s in families if _minimal(mins, s)]
            for t in families}


def cross_host(families, workdir, jobs=8, log=print):
    mins = _load(workdir, "minimised.json", {})
    db = X.DB(os.path.join(workdir, "db_cross.jsonl"))
    for t, pairs in cross_variants(families, mins).items():
        X._build_many(db, [v for _, v in pairs], workdir, jobs)
    log(f"[orders] cross: {sum(len(p) for p in cross_variants(families, mins).values())} builds")


def cross_gpu(families, workdir, replays=10, log=print):
    mins = _load(workdir, "minimised.json", {})
    doc = _load(workdir, "cross.json", {})
    for t, pairs in cross_variants(families, mins).items():
        if t in doc or not pairs:
            continue
        size = family_size(t)
        res = _eval_set(t, workdir, "db_cross.jsonl", [v for _, v in pairs], size, replays, log)
        doc[t] = {s: dict(zip(("status", "ms"), res[v.pipeline])) for s, v in pairs}
        _save(workdir, "cross.json", doc)
        log(f"[orders] cross into {t}: " + ", ".join(f"{s}:{r['status']}" for s, r in doc[t].items()))
    return doc


def write_table(workdir, families, path):
    """The committed summary: per family the best order found, its minimal form and
    that form's code object (what the benchmark times), plus the sample's census."""
    best = _load(workdir, "best.json", {})
    mins = _load(workdir, "minimised.json", {})
    doc = _load(workdir, "orders.json", {})
    fams = {}
    for f in families:
        b, m = best.get(f, {}), mins.get(f, {})
        e = dict(size=b.get("size", family_size(f)), default_ms=b.get("default_ms"))
        if b.get("order"):
            e.update(order_found=b["order"], best_ms=b.get("best_ms"), speedup=b.get("speedup"))
        if m.get("minimal") and m.get("status_minimal") == "ok" and m.get("minimal_sha256"):
            e.update(order=m["minimal"], code_sha256=m["minimal_sha256"], minimal_ms=m.get("ms_minimal"),
                     minimal_default_ms=m.get("default_ms"))
        fams[f] = e
    out = dict(seed=doc.get("seed"), count=doc.get("count"), max_len=doc.get("max_len"),
               pool_size=len(doc.get("pool", [])), census=census(workdir, families), families=fams)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    return out


# ------------------------------------------------------------------------ report --

def sample_speedups(workdir, family, n=None):
    """Speedup over the default of each sampled order in sample order (None where it
    failed), from the single exploration timing of its code object."""
    db = X.DB(os.path.join(workdir, "db.jsonl"))
    orders = load_orders(workdir)[:n]
    size = str(family_size(family))
    comp = {}
    for r in db.where(kind="compile", family=family):
        comp[r["key"]] = r.get("sha") if r["status"] == "ok" else None
    times, base = {}, None
    for r in db.where(kind="eval", family=family, status="ok"):
        t = r.get("times", {}).get(size)
        if not t:
            continue
        if r["sha"] == "default":
            base = base or t
        else:
            times.setdefault(r["sha"], t)
    if not base:
        return []
    out = []
    for o in orders:
        sha = comp.get(order_variant(family, o).key())
        out.append(base / times[sha] if sha in times else None)
    return out


def wrong_orders(workdir, families):
    """{order number: [families]} for the sampled orders whose code object gave wrong output."""
    db = X.DB(os.path.join(workdir, "db.jsonl"))
    orders = load_orders(workdir)
    out = {}
    for f in families:
        bad = {r["sha"] for r in db.where(kind="eval", family=f, status="wrong_output")}
        if not bad:
            continue
        sha_of = {}
        for r in db.where(kind="compile", family=f, status="ok"):
            sha_of[r["key"]] = r["sha"]
        for i, o in enumerate(orders):
            if sha_of.get(order_variant(f, o).key()) in bad:
                out.setdefault(i, []).append(f)
    return out


def _gm(xs):
    xs = [x for x in xs if x and x > 0]
    return math.exp(sum(math.log(x) for x in xs) / len(xs)) if xs else float("nan")


def _spearman(a, b):
    pairs = [(x, y) for x, y in zip(a, b) if x is not None and y is not None]
    if len(pairs) < 3:
        return float("nan")

    def ranks(v):
        order = sorted(range(len(v)), key=lambda i: v[i])
        r = [0.0] * len(v)
        i = 0
        while i < len(v):
            j = i
            while j + 1 < len(v) and v[order[j + 1]] == v[order[i]]:
                j += 1
            for k in range(i, j + 1):
                r[order[k]] = (i + j) / 2.0
            i = j + 1
        return r
    ra, rb = ranks([p[0] for p in pairs]), ranks([p[1] for p in pairs])
    ma, mb = statistics.fmean(ra), statistics.fmean(rb)
    num = sum((x - ma) * (y - mb) for x, y in zip(ra, rb))
    den = math.sqrt(sum((x - ma) ** 2 for x in ra) * sum((y - mb) ** 2 for y in rb))
    return num / den if den else float("nan")


STATUS_ORDER = ("ok", "no_ir", "backend_fail", "gated", "load_fail", "wrong_output", "timeout", "crashed",
                "broken_report", "error", "not_evaluated")


def report(workdir, families) -> str:
    doc = _load(workdir, "orders.json", {})
    n = doc.get("count", 0)
    cen = census(workdir, families)
    L = ["# Phase-order exploration (random LLVM pass orders on fixed kernel source)", "",
         f"{n} random orders of 1-{doc.get('max_len', MAX_LEN)} passes (seed {doc.get('seed')}), drawn uniformly "
         f"with repetition from a pool of {len(doc.get('pool', []))} passes, the same set for every family; each "
         "family at its default knobs and its benchmark size (4096, the 3D stencil 256^3); speedups are over "
         "the built-in default (`default<O3>`, same knobs).", "",
         "## Census of the sample (Sec. 3.2)", "",
         "| family | " + " | ".join(STATUS_ORDER) + " | distinct code objects |",
         "|---|" + "---:|" * (len(STATUS_ORDER) + 1)]
    tot = {}
    for f in families:
        c = cen[f]
        for k in STATUS_ORDER:
            tot[k] = tot.get(k, 0) + c.get(k, 0)
        L.append(f"| {f} | " + " | ".join(str(c.get(k, 0)) for k in STATUS_ORDER) +
                 f" | {c.get('distinct_code_objects', 0)} |")
    allv = sum(tot.values()) or 1
    L.append("| all (share) | " + " | ".join(f"{100.0 * tot[k] / allv:.1f}%" for k in STATUS_ORDER) + " | |")
    wrong = wrong_orders(workdir, families)
    if wrong:
        L += ["", "Orders whose code gave wrong output (order number in the sample: families): " +
              "; ".join(f"{i}: {', '.join(fs)}" for i, fs in sorted(wrong.items(), key=lambda kv: -len(kv[1])))
              + "."]
    sp = {f: sample_speedups(workdir, f) for f in families}
    L += ["", "## Best order of the sample, and how the sample converges (Sec. 3, 3.3)", "",
          "Best speedup over the default among the first k orders (single timings).", "",
          "| family | " + " | ".join(f"k={k}" for k in (10, 100, 500, 1000, 2000) if k <= max(n, 1)) + " |",
          "|---|" + "---:|" * len([k for k in (10, 100, 500, 1000, 2000) if k <= max(n, 1)])]
    for f in families:
        row = []
        for k in (10, 100, 500, 1000, 2000):
            if k > max(n, 1):
                continue
            vals = [x for x in sp[f][:k] if x]
            row.append(f"{max(vals):.3f}" if vals else "-")
        L.append(f"| {f} | " + " | ".join(row) + " |")
    best = _load(workdir, "best.json", {})
    mins = _load(workdir, "minimised.json", {})
    levels = _load(workdir, "phase.json", {})     # the standard levels at the default knobs (tuner phase)
    if best:
        L += ["", "## Best order per family and its minimal form (Table 1)", "",
              "Finalists re-timed with 30 replays and validated with 30 seeds; passes whose removal leaves "
              "the code object unchanged are removed on the host, then passes whose removal costs at most "
              f"{100 * MARGIN:.0f}% are removed by timing (10 replays).  `-OX`: the best of the standard "
              "levels O1, O2, O3, Os at the default knobs (the paper's -OX baseline), when measured.", "",
              "| family | best / -O3 (30 replays) | minimal / -O3 | minimal / -OX | passes in the order | "
              "same code | minimal | minimal order |",
              "|---|---:|---:|---:|---:|---:|---:|---|"]
        for f in families:
            b, m = best.get(f, {}), mins.get(f, {})
            if not b.get("order"):
                L.append(f"| {f} | no order validated | | | | | | |")
                continue
            mo = m.get("minimal")
            rmin = (f"{m['default_ms'] / m['ms_minimal']:.3f}" if m.get("default_ms") and m.get("ms_minimal")
                    else "-")
            lv = (levels.get(f) or {}).get("levels") or {}
            ox = min((t for k, t in lv.items() if t and k in ("default<O1>", "default<O2>", "default<O3>",
                                                           "default<Os>")), default=None)
            rox = f"{ox / m['ms_minimal']:.3f}" if ox and m.get("ms_minimal") else "-"
            L.append(f"| {f} | {b['speedup']:.3f} | {rmin} | {rox} | {len(b['order'])} | "
                     f"{len(m.get('same_code', [])) or '-'} | {len(mo) if mo is not None else '-'} | "
                     f"{('`' + ' '.join(p for p in mo) + '`') if mo else ('(empty)' if mo == [] else '-')} |")
    perm = _load(workdir, "permuted.json", {})
    if perm:
        L += ["", "## Permutations of each minimal order (Sec. 3.3)", "",
              "Speedup of each permutation over the minimal order itself (the same pass instances).", "",
              "| family | passes | permutations timed | failed | <=0.5 | 0.5-0.9 | 0.9-1.1 | >1.1 | worst | median |",
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
        for f in families:
            p = perm.get(f)
            if not p:
                continue
            r = p["ratios"]
            if not r:
                L.append(f"| {f} | {len(p['order'])} | 0 | {sum(p['failures'].values())} | | | | | | |")
                continue
            L.append(f"| {f} | {len(p['order'])} | {len(r)} | {sum(p['failures'].values())} | "
                     f"{sum(x <= 0.5 for x in r)} | {sum(0.5 < x < 0.9 for x in r)} | "
                     f"{sum(0.9 <= x <= 1.1 for x in r)} | {sum(x > 1.1 for x in r)} | {min(r):.3f} | "
                     f"{statistics.median(r):.3f} |")
    cross = _load(workdir, "cross.json", {})
    if cross:
        srcs = [f for f in families if _minimal(mins, f)]
        L += ["", "## Each family's minimal order on every family (Sec. 3.3)", "",
              "Rows: the family compiled; columns: whose order; entries: time of the family's own order / "
              "time with that order (1 = as fast; `x` = wrong output or failure).", "",
              "| family \\ order of | " + " | ".join(srcs) + " |", "|---|" + "---:|" * len(srcs)]
        for t in families:
            if t not in cross:
                continue
            own = (cross[t].get(t) or {}).get("ms")
            row = []
            for s in srcs:
                r = cross[t].get(s)
                if not r:
                    row.append("")
                elif r["status"] != "ok" or not r["ms"] or not own:
                    row.append("x")
                else:
                    row.append(f"{own / r['ms']:.2f}")
            L.append(f"| {t} | " + " | ".join(row) + " |")
    L += ["", "## The first 100 orders on every family (Sec. 3.3)", "",
          "Per family: how many of the first 100 orders ran correctly and how they compare with the default; "
          "then the rank correlation of the same orders' speedups between families.", "",
          "| family | valid | faster (>1.02) | same | slower (<0.98) | <=0.5 | best | median |",
          "|---|---:|---:|---:|---:|---:|---:|---:|"]
    first = {f: sp[f][:100] for f in families}
    for f in families:
        v = [x for x in first[f] if x]
        if not v:
            L.append(f"| {f} | 0 | | | | | | |")
            continue
        L.append(f"| {f} | {len(v)} | {sum(x > 1.02 for x in v)} | {sum(0.98 <= x <= 1.02 for x in v)} | "
                 f"{sum(x < 0.98 for x in v)} | {sum(x <= 0.5 for x in v)} | {max(v):.3f} | "
                 f"{statistics.median(v):.3f} |")
    L += ["", "| | " + " | ".join(families) + " |", "|---|" + "---:|" * len(families)]
    for a in families:
        L.append(f"| {a} | " + " | ".join(f"{_spearman(first[a], first[b]):.2f}" for b in families) + " |")
    return "\n".join(L) + "\n"
