"""The exploration loop (the paper's DSE, Sec. 2.3-2.4 and 3) and the feature-based
reuse experiment (Sec. 4), for one kernel family at a time.

explore   sample variants -> compile (parallel, memoised by variant) -> evaluate
          each distinct code object once on the GPU worker (memoised by code
          hash, Sec. 2.4) -> append everything to the results DB.
finalize  per size: rank by the single timing, re-time the top N with 30
          replays (Sec. 2.1), validate the fastest with 30 seeded inputs
          (Sec. 2.4), keep it only if it beats the built-in default (safe
          fallback, Sec. 4.2).
reuse     for each family, carry over the chosen variants of the K nearest
          families by code features (leave-one-out), evaluate them, keep the
          best or the default; the random-K control draws K families at random
          1000 times (Sec. 4.2).

Results live in a JSON-lines DB under the work directory, so an exploration
interrupted by a time limit resumes where it stopped.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import math
import os
import random
import time
from collections import Counter

from .. import codegen
from . import features, gate, knn, passes, space
from .evaluator import Evaluator

STATUSES = ("ok", "compile_fail", "no_output", "gated", "load_fail", "wrong_output", "timeout", "crashed",
            "broken_report", "error")


class DB:
    def __init__(self, path):
        self.path = path
        os.makedirs(os.path.dirname(path), exist_ok=True)
        self.rows = []
        if os.path.exists(path):
            with open(path) as f:
                for line in f:
                    line = line.strip()
                    if not line:
                        continue
                    try:
                        self.rows.append(json.loads(line))
                    except ValueError:
                        pass        # a truncated last line from an interrupted run

    def add(self, rec):
        rec = dict(rec, t=round(time.time(), 3))
        self.rows.append(rec)
        lead = ""
        if os.path.exists(self.path) and os.path.getsize(self.path) > 0:
            with open(self.path, "rb") as f:
                f.seek(-1, os.SEEK_END)
                lead = "" if f.read(1) == b"\n" else "\n"   # after a truncated line
        with open(self.path, "a") as f:
            f.write(lead + json.dumps(rec) + "\n")

    def where(self, **kv):
        return [r for r in self.rows if all(r.get(k) == v for k, v in kv.items())]


CODIR = None    # where code objects go (default: <workdir>/co); they can be rebuilt from the DB


def _co_path(workdir, family, sha):
    return os.path.join(CODIR or os.path.join(workdir, "co"), f"{family}_{sha[:20]}.co")


def _ensure_co(db, workdir, family, sha):
    """Path of a code object, rebuilding it from its recorded variant if it is gone."""
    p = _co_path(workdir, family, sha)
    if os.path.exists(p):
        return p
    var = _variant_of(db, family, sha)
    if var is not None:
        rec = _build(space.Variant.from_json(var), workdir)
        if rec["status"] == "ok" and rec["sha"] == sha:
            return p
    return None


def _build_many(db, variants, workdir, jobs):
    """Compile records for `variants` (memoised through the DB), misses in parallel."""
    recs = [None] * len(variants)
    miss = []
    for i, v in enumerate(variants):
        for r in db.where(kind="compile", key=v.key(), status="ok"):
            if os.path.exists(_co_path(workdir, v.family, r["sha"])):
                recs[i] = r
                break
        else:
            miss.append(i)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for i, rec in zip(miss, ex.map(lambda i: _build(variants[i], workdir), miss)):
            db.add(rec)
            recs[i] = rec
    return recs


def _build(v: space.Variant, workdir):
    t0 = time.time()
    try:
        b = codegen.compile_variant(v.family, v.knobs, v.pipeline, v.llc_flags, timeout=180,
                                    opt_flags=v.opt_flags)
    except codegen.CompileError as e:
        status = "no_output" if "no optimised IR" in str(e) else "compile_fail"
        return dict(kind="compile", family=v.family, key=v.key(), variant=v.to_json(), status=status,
                    stage=e.stage, detail=str(e)[-300:], seconds=round(time.time() - t0, 2))
    except Exception as e:      # noqa: BLE001
        return dict(kind="compile", family=v.family, key=v.key(), variant=v.to_json(), status="compile_fail",
                    stage="driver", detail=f"{type(e).__name__}: {e}"[-300:], seconds=round(time.time() - t0, 2))
    reason = gate.check(b.code)
    if reason:
        # built, but never handed to the GPU (see tuner/gate.py)
        return dict(kind="compile", family=v.family, key=v.key(), variant=v.to_json(), status="gated",
                    stage="gate", sha=b.code_hash, detail=reason[-300:], seconds=round(time.time() - t0, 2))
    p = _co_path(workdir, v.family, b.code_hash)
    os.makedirs(os.path.dirname(p), exist_ok=True)
    if not os.path.exists(p):
        with open(p, "wb") as f:
            f.write(b.code)
    return dict(kind="compile", family=v.family, key=v.key(), variant=v.to_json(), status="ok", sha=b.code_hash,
                seconds=round(time.time() - t0, 2))


def _evaluate(ev, db, family, sha, path, sizes, cutoff, timeout, replays=1, seeds=1, validate=True):
    res = ev.request(dict(op="eval", code=path, validate=validate, seeds=seeds, time=True,
                          sizes=sizes, replays=replays, cutoff=cutoff), timeout=timeout)
    rec = dict(kind="eval", family=family, sha=sha, status=res.get("status", "error"),
               times=res.get("times", {}), err=res.get("err"), detail=res.get("detail", ""),
               replays=replays)
    db.add(rec)
    return rec


class WorkerFailure(RuntimeError):
    """A candidate killed or hung its worker; the exploration stops (stop_on_failure)."""


def explore(family, workdir, samples=500, seed=5500, sizes=(256, 512, 1000, 2048, 4096), jobs=8,
            eval_timeout=120.0, log=print, max_minutes=None, pool=None, make_evaluator=None, build=None,
            variants=None, stop_on_failure=False):
    """Compile and evaluate a family's sample (the knob sample, or `variants`: the
    default first).  With `stop_on_failure`, the first candidate whose worker dies or
    hangs ends the exploration (WorkerFailure): it may have faulted the GPU."""
    t_start = time.time()
    db = DB(os.path.join(workdir, "db.jsonl"))
    if variants is None:
        pool = pool if pool is not None else passes.load_pool()
        variants = [space.default_variant(family)] + space.sample_variants(family, pool, samples, seed)
    compiled = {r["key"]: r for r in db.where(kind="compile", family=family)}
    evaluated = {r["sha"]: r for r in db.where(kind="eval", family=family)}
    build = build or _build
    ev = (make_evaluator or (lambda: Evaluator(family, sizes, log=log,
                                               stderr_path=os.path.join(workdir, f"worker_{family}.err"))))()
    log(f"[explore] {family}: {len(variants)} variants, {len(compiled)} compiled and "
        f"{len(evaluated)} code objects evaluated before")
    if "default" not in evaluated:
        evaluated["default"] = _evaluate(ev, db, family, "default", "default", list(sizes), None, 600,
                                         replays=3, validate=False)
    base = evaluated["default"].get("times", {})
    log(f"[explore] {family} default ms/launch: " + ", ".join(f"{k}:{v:.4f}" for k, v in base.items()))
    cutoff = {k: 20.0 * v for k, v in base.items()}
    todo = [v for v in variants if v.key() not in compiled]
    done = 0

    def eval_if_new(rec):
        nonlocal done
        if rec["status"] != "ok" or rec["sha"] in evaluated:
            return
        e = _evaluate(ev, db, family, rec["sha"], _co_path(workdir, family, rec["sha"]), list(sizes), cutoff,
                      eval_timeout)
        evaluated[rec["sha"]] = e
        done += 1
        if stop_on_failure and e["status"] in ("crashed", "timeout"):
            ev.close()
            raise WorkerFailure(f"{family}: candidate {rec['sha'][:12]} {e['status']}; exploration stopped")
        big = str(max(sizes))
        tb = e["times"].get(big)
        log(f"[explore] {family} #{done} {e['status']} sha={rec['sha'][:10]} "
            f"t{big}={'%.4f' % tb if tb else '-'} pipeline={rec['variant']['pipeline'][:48]}")

    # code objects compiled in an earlier (interrupted) run, or on another machine,
    # but never evaluated
    for rec in list(compiled.values()):
        if rec["status"] == "ok" and rec["sha"] not in evaluated:
            if _ensure_co(db, workdir, family, rec["sha"]) is None:
                continue
            eval_if_new(rec)
            if max_minutes and time.time() - t_start > 60 * max_minutes:
                log(f"[explore] {family}: time limit reached, stopping (resumable)")
                ev.close()
                return census(db, family, {v.key() for v in variants})
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(build, v, workdir) for v in todo]
        for fut in cf.as_completed(futs):
            rec = fut.result()
            db.add(rec)
            compiled[rec["key"]] = rec
            if rec["status"] != "ok":
                log(f"[explore] {family} {rec['status']} at {rec.get('stage')}: {rec['variant']['pipeline'][:48]}")
            eval_if_new(rec)
            if max_minutes and time.time() - t_start > 60 * max_minutes:
                log(f"[explore] {family}: time limit reached, stopping (resumable)")
                for f_ in futs:
                    f_.cancel()
                break
    ev.close()
    return census(db, family, {v.key() for v in variants})


def census(db, family, keys=None):
    """Outcome counts over the family's sampled variants (compile failures and
    evaluation outcomes of their code objects; the paper's Sec. 3.2 census).
    One count per variant (its latest compile record); `keys` restricts the
    count to one sample."""
    latest = {}
    for r in db.where(kind="compile", family=family):
        if keys is None or r["key"] in keys:
            latest[r["key"]] = r
    comp = list(latest.values())
    evals = {r["sha"]: r for r in db.where(kind="eval", family=family)}
    c = Counter()
    for r in comp:
        if r["status"] != "ok":
            c[r["status"]] += 1
        else:
            c[evals.get(r["sha"], {}).get("status", "not_evaluated")] += 1
    c["distinct_code_objects"] = len({r["sha"] for r in comp if r["status"] == "ok"})
    c["variants"] = len(comp)
    return dict(c)


def _variant_of(db, family, sha):
    for r in db.where(kind="compile", family=family, status="ok"):
        if r.get("sha") == sha:
            return r["variant"]
    return None


def finalize(family, workdir, sizes=(256, 512, 1000, 2048, 4096), top=10, replays=30, seeds=30,
             eval_timeout=300.0, log=print, margin=0.03, exclude=()):
    """Choose the variant per size bucket (or the default) and return table entries.

    A candidate replaces the default only if its re-timed launch is at least
    `margin` faster: microsecond launches differ by a few percent from one
    timing to the next, and a table entry has to pay for itself.  Code objects
    whose hashes are in `exclude` do not compete."""
    db = DB(os.path.join(workdir, "db.jsonl"))
    evals = [r for r in db.where(kind="eval", family=family, status="ok")
             if r["sha"] != "default" and r["sha"] not in set(exclude)]
    ev = Evaluator(family, sizes, log=log, stderr_path=os.path.join(workdir, f"worker_{family}.err"))
    entries = []
    from ..api import Context
    for size in sizes:
        key = str(size)
        ranked = sorted((r for r in evals if key in r.get("times", {})), key=lambda r: r["times"][key])
        uniq, seen = [], set()
        for r in ranked:
            if r["sha"] not in seen:
                seen.add(r["sha"])
                uniq.append(r)
        cands = uniq[:top]
        d = _evaluate(ev, db, family, "default", "default", [size], None, eval_timeout, replays=replays,
                      validate=False)
        t_def = d["times"].get(key, math.inf)
        timed = []
        for r in cands:
            path = _ensure_co(db, workdir, family, r["sha"])
            if path is None:
                continue
            e = _evaluate(ev, db, family, r["sha"], path, [size], None,
                          eval_timeout, replays=replays, validate=False)
            if e["status"] == "ok" and key in e["times"]:
                timed.append((e["times"][key], r["sha"]))
        timed.sort()
        chosen = None
        for t, sha in timed:
            if t >= t_def * (1.0 - margin):
                break
            v = _evaluate(ev, db, family, sha, _ensure_co(db, workdir, family, sha), [], None, eval_timeout,
                          validate=True, seeds=seeds)
            v_ok = v["status"] == "ok"
            log(f"[finalize] {family}/{size}: {sha[:10]} {t:.4f} ms vs default {t_def:.4f} ms; "
                f"{seeds}-seed validation {'passed' if v_ok else 'FAILED'}")
            if v_ok:
                chosen = (t, sha)
                break
        bucket = Context.size_bucket(size)
        if chosen is None:
            entries.append(dict(family=family, bucket=bucket, size=size, is_default=True,
                                knobs=space.default_knobs(family), pipeline=codegen.DEFAULT_PIPELINE,
                                default_ms=t_def, tuned_ms=t_def, speedup=1.0))
            continue
        t, sha = chosen
        var = _variant_of(db, family, sha)
        entries.append(dict(family=family, bucket=bucket, size=size, is_default=False, knobs=var["knobs"],
                            pipeline=var["pipeline"], llc_flags=var.get("llc_flags", ["-O3"]),
                            opt_flags=var.get("opt_flags", []), code_sha256=sha,
                            default_ms=t_def, tuned_ms=t, speedup=t_def / t))
    ev.close()
    with open(os.path.join(workdir, f"table_{family}.json"), "w") as f:
        json.dump(entries, f, indent=1)
    return entries


# the one-launch forms (FUSE = 1) of the transposed matvec, the pair and the column
# statistics: wavefronts stacked over the rows of one strip, the last block of each
# group folding the partials; the grid `refine` adds to a table measured without them
ONE_LAUNCH_GRID = {
    "gemv_t": [dict(ROWS=r, WAVES=w, VEC=v, UNROLL=u, ORDER=0, FUSE=1) for r in (128, 256, 512)
               for w in (4, 8) for v in (1, 2, 4) for u in (4, 8, 16)]
              + [dict(ROWS=r, WAVES=w, VEC=v, UNROLL=16, ORDER=o, NTL=1) for r in (16, 32, 64, 128)
                 for w in (2, 4, 8) for v in (1, 2, 4) for o in (0, 1)],     # non-temporal, two launches
    "gemv_pair": [dict(ROWS=r, WAVES=w, VEC=v, UNROLL=u, ORDER=0, FUSE=1) for r in (128, 256, 512)
                  for w in (4, 8) for v in (1, 2, 4) for u in (4, 8, 16)]
                 + [dict(ROWS=r, WAVES=w, VEC=v, UNROLL=16, ORDER=o, NTL=1) for r in (16, 32, 64, 128)
                    for w in (2, 4, 8) for v in (1, 2, 4) for o in (0, 1)],
    "gemv": [dict(ROWS=r, WAVES=w, VEC=4, UNROLL=u, USE_LDS=l, ORDER=0, NTL=1) for r in (1, 2, 4)
             for w in (2, 4, 8) for u in (1, 2, 4) for l in (0, 1)],
    "colstats": [dict(VEC=v, WAVES=w, ROWS=r, ORDER=0, FUSE=1) for v in (1, 2, 4) for w in (4, 8)
                 for r in (128, 256, 512)]
                + [dict(VEC=v, WAVES=w, ROWS=r, ORDER=o, NTL=ntl, MG=1) for v in (1, 2, 4) for w in (4, 8)
                   for r in (16, 32, 64, 128) for o in (0, 1) for ntl in (0, 1)],   # the one-pass merge
}


def _stencil_grids():
    """Structured grids around the stencils' best sampled variants: the 3D stencil's
    staged form with tiles 128 or 256 columns wide (256 = a whole row of the 256^3
    volume: no x halo), 16 or 32 rows, 8-32 planes per block and one or two planes
    fetched ahead; the 2D stencil's
    register-window form with 256-1024-column tiles."""
    g3 = []
    for tx, vec in ((32, 4), (64, 2), (64, 4), (128, 1), (128, 2)):
        for ty, yr in ((2, 8), (4, 4), (8, 2), (4, 8), (8, 4)):
            for rows in (8, 16, 32):
                for order in (0, 1, 2):
                    for pf in (1, 2):
                        g3.append(dict(TX=tx, VEC=vec, TY=ty, YR=yr, ROWS=rows, USE_LDS=2, UNROLL=1, ORDER=order,
                                       PF=pf))
    g2 = [dict(TX=tx, VEC=vec, TY=ty, ROWS=rows, UNROLL=1, USE_LDS=0, ORDER=order)
          for tx in (64, 128, 256) for vec in (2, 4) for ty in (1, 2, 4) for rows in (8, 16, 32)
          for order in (0, 2)]
    return {"conv3d": g3, "conv2d": g2, "gemm_f32": _gemm32_grid(), "syrk_f32": _syrk32_grid()}


def _syrk32_grid():
    """The FP32 rank-k product of the correlation with the interleaved k loop of full
    tiles (IL; IL = 2 for sample counts that are not a multiple of the step): 32-128-wide
    triangle tiles, 1-16 wavefronts, k steps 16-128 deep (the deep ones for small sample
    counts: a 256-sample problem in two to four steps), the row-order and the XCD-aware
    rasters."""
    return [dict(BT=bt, BK=bk, WAVES_M=wm, WAVES_N=wn, VEC=4, STAGES=2, ORDER=order, IL=il)
            for il in (1, 2) for bt in (32, 64, 96, 128) for bk in (16, 32, 64, 128)
            for wm, wn in ((1, 1), (1, 2), (2, 1), (2, 2), (2, 4), (4, 2), (4, 4)) for order in (0, 2)] + \
        [dict(BT=bt, BK=bk, WAVES_M=wm, WAVES_N=wn, VEC=4, STAGES=2, ORDER=order, IL=3)
         for bt in (32, 64) for bk in (16, 32)
         for wm, wn in ((1, 1), (1, 2), (2, 1), (2, 2), (2, 4), (4, 2), (4, 4)) for order in (0, 2)]


def _gemm32_grid():
    """The FP32 GEMM around its sampled optimum: 128- and 256-wide tiles, 4 or 8
    wavefronts, 16x16 or 32x32 MFMA blocks, k steps 16-64 deep (64 with the fragments
    read four k at a time), one or two LDS stages, row padding 4 or 8 floats; and the
    same tiles with the interleaved k loop of full tiles (IL)."""
    out = []
    for bm, bn in ((128, 128), (256, 128), (128, 256), (256, 256)):
        for wm, wn in ((1, 1), (2, 1), (1, 2), (2, 2), (4, 2), (2, 4)):
            for bk, fc in ((16, 0), (32, 0), (32, 4), (64, 4)):
                for lds in (1, 2):
                    for pad in (4, 8):
                        for mf in (16, 32):
                            if mf == 16 and pad == 4 and fc == 0:
                                continue        # the sampled space
                            out.append(dict(BM=bm, BN=bn, WAVES_M=wm, WAVES_N=wn, BK=bk, USE_LDS=lds, LDS_PAD=pad,
                                            MF=mf, FC=fc, VEC=4, UNROLL=1, ORDER=3))
            # the interleaved k loop of full tiles (two LDS stages, whole-fragment reads)
            for bk in (16, 32):
                for pad in (4, 8):
                    for mf in (16, 32):
                        out.append(dict(BM=bm, BN=bn, WAVES_M=wm, WAVES_N=wn, BK=bk, USE_LDS=2, LDS_PAD=pad,
                                        MF=mf, FC=0, IL=1, VEC=4, UNROLL=1, ORDER=3))
    # small problems with full tiles: the interleaved loop with 32- and 64-wide tiles and
    # k steps up to 128 deep (a 256-deep product in two to eight steps)
    for bm in (32, 64):
        for bn in (32, 64):
            for wm, wn in ((1, 1), (2, 1), (1, 2), (2, 2)):
                for bk in (32, 64, 128):
                    for pad in (4, 8):
                        out.append(dict(BM=bm, BN=bn, WAVES_M=wm, WAVES_N=wn, BK=bk, USE_LDS=2, LDS_PAD=pad,
                                        MF=16, FC=0, IL=1, VEC=4, UNROLL=1, ORDER=3))
    # K not a multiple of the k step (a masked last tile): 32-128-wide tiles
    for bm in (32, 64, 128):
        for bn in (32, 64, 128):
            for wm, wn in ((1, 1), (2, 1), (1, 2), (2, 2), (2, 4), (4, 2)):
                for bk in (32, 64):
                    out.append(dict(BM=bm, BN=bn, WAVES_M=wm, WAVES_N=wn, BK=bk, USE_LDS=2, LDS_PAD=8,
                                    MF=16, FC=0, IL=2, VEC=4, UNROLL=1, ORDER=3))
    # small problems: fragments loaded straight from memory without branches (DK), the k
    # loop unrolled 2-8 deep so that several k tiles' loads are in flight at once
    for bm in (16, 32, 64):
        for bn in (16, 32, 64):
            for wm, wn in ((1, 1), (1, 2), (2, 1), (2, 2)):
                for bk in (16, 32):
                    for u in (2, 4, 8):
                        out.append(dict(BM=bm, BN=bn, WAVES_M=wm, WAVES_N=wn, BK=bk, USE_LDS=0, DK=1, UNROLL=u,
                                        VEC=4, ORDER=3))
    return out


REFINE_GRIDS = dict(ONE_LAUNCH_GRID, **_stencil_grids())


def refine(family, workdir, table_path, grid, sizes=(256, 512, 1000, 2048, 4096), top=5, replays=30, seeds=30,
           eval_timeout=300.0, log=print, margin=0.03, jobs=8, tag="refined"):
    """Extend a finished table along new knob settings without a new exploration.

    Every setting of `grid` (knob overrides of the family's default, -O3) is compiled,
    gated, timed once per size; per size the `top` fastest, the table's current entry
    and the default are re-timed with `replays` replays, and the fastest candidate
    replaces the entry only if it beats the re-timed entry by `margin` and passes the
    `seeds`-seed validation (as in finalize).  Entries are rewritten in `table_path`
    in place; the default's time and the speedups are the re-timed ones."""
    from .. import tuned
    from ..api import Context
    db = DB(os.path.join(workdir, "db.jsonl"))
    variants = [space.Variant(family, dict(space.default_knobs(family), **g), codegen.DEFAULT_PIPELINE)
                for g in grid]
    variants = [v for v in variants if space.valid(family, v.knobs)]
    recs = _build_many(db, variants, workdir, jobs)
    cands = [(v, r) for v, r in zip(variants, recs) if r["status"] == "ok"]
    log(f"[refine] {family}: {len(cands)} of {len(variants)} grid settings built and gated")
    with open(table_path) as f:
        doc = json.load(f)
    entries = doc["entries"]
    ev = Evaluator(family, sizes, log=log, stderr_path=os.path.join(workdir, f"worker_{family}.err"))
    changed = 0
    try:
        for size in sizes:
            key = str(size)
            bucket = Context.size_bucket(size)
            idx = [i for i, e in enumerate(entries) if e["family"] == family and int(e["bucket"]) == bucket]
            if len(idx) != 1:
                log(f"[refine] {family}/{size}: no single table entry, skipped")
                continue
            cur = entries[idx[0]]
            once = []
            for v, r in cands:
                e = _evaluate(ev, db, family, r["sha"], _co_path(workdir, family, r["sha"]), [size], None,
                              eval_timeout, validate=True, seeds=1)
                if e["status"] == "ok" and key in e["times"]:
                    once.append((e["times"][key], r["sha"], v))
            once.sort(key=lambda t: t[0])
            d = _evaluate(ev, db, family, "default", "default", [size], None, eval_timeout, replays=replays,
                          validate=False)
            t_def = d["times"].get(key, math.inf)
            t_cur = t_def
            if not cur.get("is_default"):
                code = tuned.code_for(cur)
                if code is None:
                    log(f"[refine] {family}/{size}: the table entry does not reproduce, skipped")
                    continue
                p = _co_path(workdir, family, cur["code_sha256"])
                os.makedirs(os.path.dirname(p), exist_ok=True)
                with open(p, "wb") as f:
                    f.write(code)
                c = _evaluate(ev, db, family, cur["code_sha256"], p, [size], None, eval_timeout,
                              replays=replays, validate=False)
                t_cur = c["times"].get(key, math.inf)
            timed = []
            for _, sha, v in once[:top]:
                e = _evaluate(ev, db, family, sha, _co_path(workdir, family, sha), [size], None, eval_timeout,
                              replays=replays, validate=False)
                if e["status"] == "ok" and key in e["times"]:
                    timed.append((e["times"][key], sha, v))
            timed.sort(key=lambda t: t[0])
            log(f"[refine] {family}/{size}: default {t_def:.4f} ms, table {t_cur:.4f} ms, best of grid "
                + (f"{timed[0][0]:.4f} ms {timed[0][2].knobs}" if timed else "-"))
            if not timed or timed[0][0] >= t_cur * (1.0 - margin):
                entries[idx[0]] = dict(cur, default_ms=t_def, tuned_ms=t_cur, speedup=t_def / t_cur)
                continue
            t, sha, v = timed[0]
            val = _evaluate(ev, db, family, sha, _co_path(workdir, family, sha), [], None, eval_timeout,
                            validate=True, seeds=seeds)
            if val["status"] != "ok":
                log(f"[refine] {family}/{size}: {sha[:10]} failed the {seeds}-seed validation")
                continue
            entries[idx[0]] = dict(family=family, bucket=bucket, size=size, is_default=False, knobs=v.knobs,
                                   pipeline=v.pipeline, llc_flags=list(v.llc_flags), opt_flags=list(v.opt_flags),
                                   code_sha256=sha, default_ms=t_def, tuned_ms=t, speedup=t_def / t,
                                   source="one-launch grid" if v.knobs.get("FUSE", 0) else tag)
            changed += 1
    finally:
        ev.close()
    doc["entries"] = entries
    with open(table_path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    return changed


def upgrade_accepts(t_cur, t_new, margin, gain):
    """Whether a rebuilt entry (t_new ms) replaces the entry (t_cur ms): both timed (a size
    without a workload times as inf), and not slower by more than `margin` (a capability)
    or, with `gain`, faster by at least `margin` (a knob that is there for speed alone)."""
    if not (math.isfinite(t_cur) and math.isfinite(t_new)):
        return False
    return t_new <= t_cur * ((1.0 - margin) if gain else (1.0 + margin))


def upgrade(family, workdir, table_path, extra, sizes=(256, 512, 1000, 2048, 4096), replays=30, seeds=30,
            eval_timeout=300.0, log=print, margin=0.03, jobs=8, tag="upgraded", gain=False):
    """Rebuild each non-default table entry with the knobs `extra` added, keeping its
    pipeline and flags, and take the rebuilt code object if, re-timed with `replays`
    replays beside the entry, it passes the `seeds`-seed validation and is not slower
    than the entry by more than `margin` (a capability that leaves the entry's own
    launches unchanged, e.g. EPI) or, with `gain`, is faster by at least `margin` (a
    knob that is there for speed alone, e.g. NTL)."""
    from .. import tuned
    from ..api import Context
    db = DB(os.path.join(workdir, "db.jsonl"))
    with open(table_path) as f:
        doc = json.load(f)
    entries = doc["entries"]
    ev = Evaluator(family, sizes, log=log, stderr_path=os.path.join(workdir, f"worker_{family}.err"))
    changed = 0
    try:
        for size in sizes:
            key = str(size)
            bucket = Context.size_bucket(size)
            idx = [i for i, e in enumerate(entries) if e["family"] == family and int(e["bucket"]) == bucket]
            # an entry that kept the default is a candidate only for a knob that must gain:
            # then the family's default, with the knobs added, is timed against the default
            if len(idx) != 1 or (entries[idx[0]].get("is_default") and not gain):
                continue
            cur = entries[idx[0]]
            v = space.Variant(family, dict(cur["knobs"], **extra), cur["pipeline"],
                              tuple(cur.get("llc_flags", ["-O3"])), tuple(cur.get("opt_flags", [])))
            if not space.valid(family, dict(space.default_knobs(family), **v.knobs)):
                log(f"[upgrade] {family}/{size}: {extra} does not combine with the entry's knobs")
                continue
            rec = _build_many(db, [v], workdir, jobs)[0]
            if cur.get("is_default"):
                base = _build_many(db, [space.Variant(family, space.default_knobs(family), codegen.DEFAULT_PIPELINE)],
                                   workdir, jobs)[0]
                cur_sha = base["sha"] if base["status"] == "ok" else None
                code = True if cur_sha else None
            else:
                cur_sha = cur["code_sha256"]
                code = tuned.code_for(cur)
            if rec["status"] != "ok" or code is None:
                log(f"[upgrade] {family}/{size}: not built ({rec['status']}) or the entry does not reproduce")
                continue
            p = _co_path(workdir, family, cur_sha)
            if code is not True:
                os.makedirs(os.path.dirname(p), exist_ok=True)
                with open(p, "wb") as f:
                    f.write(code)
            c = _evaluate(ev, db, family, cur_sha, p, [size], None, eval_timeout, replays=replays,
                          validate=False)
            n = _evaluate(ev, db, family, rec["sha"], _co_path(workdir, family, rec["sha"]), [size], None,
                          eval_timeout, replays=replays, validate=False)
            t_cur, t_new = c["times"].get(key, math.inf), n["times"].get(key, math.inf)
            log(f"[upgrade] {family}/{size}: entry {t_cur:.4f} ms, with {extra} {t_new:.4f} ms")
            if not upgrade_accepts(t_cur, t_new, margin, gain):
                continue
            val = _evaluate(ev, db, family, rec["sha"], _co_path(workdir, family, rec["sha"]), [], None,
                            eval_timeout, validate=True, seeds=seeds)
            if val["status"] != "ok":
                log(f"[upgrade] {family}/{size}: failed the {seeds}-seed validation")
                continue
            entries[idx[0]] = dict(cur, knobs=v.knobs, code_sha256=rec["sha"], tuned_ms=t_new,
                                   speedup=cur["default_ms"] / t_new, source=tag, is_default=False,
                                   llc_flags=list(v.llc_flags), opt_flags=list(v.opt_flags))
            changed += 1
    finally:
        ev.close()
    doc["entries"] = entries
    with open(table_path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    return changed


def reuse(families, workdir, sizes=(256, 512, 1000, 2048, 4096), ks=(1, 3), trials=1000, replays=10,
          eval_timeout=300.0, jobs=8, log=print, seed=5500):
    """Feature-based reuse with leave-one-out, and the random-K control."""
    db = DB(os.path.join(workdir, "db.jsonl"))
    tables = {}
    for fam in families:
        with open(os.path.join(workdir, f"table_{fam}.json")) as f:
            tables[fam] = {e["size"]: e for e in json.load(f)}
    feats = features.family_features(families)
    vecs = knn.vectors(feats, features.FEATURE_NAMES)

    def best_variant(fam, size):
        e = tables[fam][size]
        return space.Variant(fam, e["knobs"], e["pipeline"], tuple(e.get("llc_flags", ["-O3"])),
                             tuple(e.get("opt_flags", [])))

    times = {}      # (target, source, size) -> ms or None
    carried = {}    # (target, source, size) -> (transferred variant, code sha)
    for target in families:
        todo = []
        for source in families:
            if source == target:
                continue
            for size in sizes:
                v = space.transfer(best_variant(source, size), target)
                todo.append((source, size, v))
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            built = _build_many(db, [t[2] for t in todo], workdir, jobs)
        ev = Evaluator(target, sizes, log=log, stderr_path=os.path.join(workdir, f"worker_{target}.err"))
        memo = {}
        for (source, size, v), rec in zip(todo, built):
            if rec["status"] != "ok":
                times[(target, source, size)] = None
                continue
            carried[(target, source, size)] = (v, rec["sha"])
            k = (rec["sha"], size)
            if k not in memo:
                e = _evaluate(ev, db, target, rec["sha"], _co_path(workdir, target, rec["sha"]), [size], None,
                              eval_timeout, replays=replays, validate=True, seeds=1)
                memo[k] = e["times"].get(str(size)) if e["status"] == "ok" else None
            times[(target, source, size)] = memo[k]
        ev.close()
        log(f"[reuse] {target}: {len(todo)} transfers evaluated ({len(memo)} distinct)")

    def t_def(fam, size):
        return tables[fam][size]["default_ms"]

    items = [(f, s) for f in families for s in sizes]
    out = {"nearest": {f: knn.nearest(f, vecs, max(ks)) for f in families}}
    for k in ks:
        sp = []
        for f, s in items:
            srcs = knn.nearest(f, vecs, k)
            tt = knn.best_of([times.get((f, x, s)) for x in srcs], t_def(f, s))
            sp.append(t_def(f, s) / tt)
        out[f"cosine_k{k}"] = knn.geomean(sp)
        rng = random.Random(seed + k)
        vals = []
        for _ in range(trials):
            sp = []
            for f, s in items:
                others = [x for x in families if x != f]
                srcs = rng.sample(others, min(k, len(others)))
                tt = knn.best_of([times.get((f, x, s)) for x in srcs], t_def(f, s))
                sp.append(t_def(f, s) / tt)
            vals.append(knn.geomean(sp))
        out[f"random_k{k}"] = sum(vals) / len(vals)
    out["tuned"] = knn.geomean([tables[f][s]["speedup"] for f, s in items])
    # the assignment each K makes: per (family, size) the fastest of the K
    # carried-over variants, or the default when none beats it
    from ..api import Context
    assign = []
    for k in ks:
        for f, s in items:
            srcs = knn.nearest(f, vecs, k)
            cands = sorted((times[(f, x, s)], x) for x in srcs
                           if times.get((f, x, s)) is not None and 0 < times[(f, x, s)] < t_def(f, s))
            e = dict(family=f, size=s, bucket=Context.size_bucket(s), k=k, sources=srcs, default_ms=t_def(f, s))
            if cands:
                t, x = cands[0]
                v, sha = carried[(f, x, s)]
                e.update(is_default=False, source=x, ms=t, code_sha256=sha, **v.to_json())
            else:
                e.update(is_default=True, ms=t_def(f, s))
            assign.append(e)
    out["assign"] = assign
    out["transfers"] = {f"{t}<-{s}@{z}": v for (t, s, z), v in times.items()}
    with open(os.path.join(workdir, "reuse.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


def write_table(families, workdir, path, extra=None):
    """Merge the per-family tables into the package's tuning table."""
    entries = []
    for fam in families:
        p = os.path.join(workdir, f"table_{fam}.json")
        if os.path.exists(p):
            with open(p) as f:
                entries += json.load(f)
    doc = dict(version=1, arch=codegen.ARCH, entries=entries)
    rp = os.path.join(workdir, "reuse.json")
    if os.path.exists(rp):
        with open(rp) as f:
            r = json.load(f)
        doc["reuse"] = [e for e in r.get("assign", []) if e["family"] in families]
        doc["reuse_summary"] = {k: v for k, v in r.items() if k not in ("assign", "transfers")}
    if extra:
        doc.update(extra)
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    return doc
