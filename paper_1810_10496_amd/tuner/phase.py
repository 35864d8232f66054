"""Phase-order analysis of the knob exploration (the paper's Sec. 3.1 and 3.3
experiments, carried over to the pipelines that exploration samples).

The knob exploration pairs each knob draw with a standard pipeline or the flags of
its passes (random phase orders on fixed source are `tuner.orders`), so these
experiments take these forms:

  levels     the default knobs under each standard level (O1, O2, O3, Os, Oz),
             timed at one size: how far the levels are apart (the paper finds
             that they rarely differ, Sec. 3.1);
  minimise   each family's tuned variant at that size, when its pipeline
             carries flags: re-timed as it is, without each flag in turn and
             without any -- the paper minimises its best sequences by removing
             passes that change nothing (Table 1); a flag whose removal costs
             more than the noise margin is part of the minimal set;
  first100   (from the exploration database, no GPU) the first 100 sampled
             variants' speedups over the default at the largest size, the
             paper's scatter of its first 100 sequences (Sec. 3.3).

Permutations of a best sequence (the paper's last experiment) apply to the
random orders (`tuner.orders`): a standard pipeline's pass order is fixed, and
flags have none.

    python -m paper_1810_10496_amd.tuner phase --workdir D --families F --size 4096

writes D/phase.json; its evaluations go to D/db_phase.jsonl, apart from the
exploration database, whose rows the finalisation reads.
"""
from __future__ import annotations

import json
import os
import statistics

from .. import workloads as W
from . import explore as X, space
from .evaluator import Evaluator

MARGIN = 0.02      # a flag is kept when removing it costs more than this


def level_variants(family: str) -> list[tuple[str, space.Variant]]:
    k = space.default_knobs(family)
    return [(lvl, space.Variant(family, dict(k), lvl)) for lvl in space.STANDARD]


def minimise_variants(entry: dict) -> list[tuple[str, space.Variant]]:
    """The tuned variant, the variant without each of its flags, and without all of them
    (empty when the variant carries no flags beyond -O3)."""
    fam, knobs, pipe = entry["family"], dict(entry.get("knobs", {})), entry.get("pipeline", "default<O3>")
    of = tuple(entry.get("opt_flags", []))
    lf = tuple(entry.get("llc_flags", ["-O3"]))
    extra = [f for f in lf if f != "-O3"]
    if not of and not extra:
        return []
    out = [("tuned", space.Variant(fam, knobs, pipe, lf, of))]
    for f in of:
        out.append((f"without {f}", space.Variant(fam, knobs, pipe, lf, tuple(x for x in of if x != f))))
    for f in extra:
        out.append((f"without {f}", space.Variant(fam, knobs, pipe, tuple(x for x in lf if x != f), of)))
    out.append(("without flags", space.Variant(fam, knobs, pipe, ("-O3",), ())))
    return out


def minimal_flags(times: dict) -> list[str]:
    """Flags whose removal slows the tuned variant by more than MARGIN."""
    t = times.get("tuned")
    if not t:
        return []
    return [tag[len("without "):] for tag, v in times.items()
            if tag.startswith("without -") and v and v > t * (1.0 + MARGIN)]


def run(families, workdir, table_entries, size, replays=10, jobs=8, log=print, make_evaluator=None,
        build=None, build_only=False):
    db = X.DB(os.path.join(workdir, "db_phase.jsonl"))
    out_path = os.path.join(workdir, "phase.json")
    doc = json.load(open(out_path)) if os.path.exists(out_path) else {}
    for fam in families:
        fsize = W.CONV3D_SIZE if fam == "conv3d" else int(size)     # the 3D stencil has one grid
        entry = next((e for e in table_entries if e["family"] == fam and int(e["size"]) == fsize), None)
        lv = level_variants(fam)
        mv = minimise_variants(entry) if entry and not entry.get("is_default") else []
        tagged = [("level", t, v) for t, v in lv] + [("minimise", t, v) for t, v in mv]
        variants = [v for _, _, v in tagged]
        if build:
            recs = [build(v, workdir) for v in variants]
            for r in recs:
                db.add(r)
        else:
            recs = X._build_many(db, variants, workdir, jobs)
        bad = [r for r in recs if r["status"] != "ok"]
        log(f"[phase] {fam}: {len(variants)} variants, {len(bad)} failed to build")
        if build_only:
            continue
        ev = (make_evaluator or (lambda: Evaluator(fam, [fsize], log=log,
                                                   stderr_path=os.path.join(workdir, f"worker_{fam}.err"))))()
        res = {"size": fsize, "levels": {}, "minimise": {}, "status": {}}
        for (kind, tag, v), rec in zip(tagged, recs):
            if rec["status"] != "ok":
                res["status"][f"{kind}:{tag}"] = rec["status"]
                continue
            e = X._evaluate(ev, db, fam, rec["sha"], X._co_path(workdir, fam, rec["sha"]), [fsize], None, 300,
                            replays=replays, validate=True)
            t = e["times"].get(str(fsize)) if e["status"] == "ok" else None
            if e["status"] != "ok":
                res["status"][f"{kind}:{tag}"] = e["status"]
            res["levels" if kind == "level" else "minimise"][tag] = t
        ev.close()
        if mv:
            res["flags"] = [t[len("without "):] for t, _ in mv if t.startswith("without -")]
            res["minimal"] = minimal_flags(res["minimise"])
        doc[fam] = res
        log(f"[phase] {fam}: levels " + ", ".join(f"{k} {v:.4f}" for k, v in res["levels"].items() if v)
            + (f"; minimal flags {res.get('minimal')}" if mv else ""))
        with open(out_path, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
    return doc


def _sample_speedups(db, family, size, samples, seed, pool, n):
    """Speedup over the default at `size` of each of the first `n` sampled variants, in
    sample order (None where a variant did not compile or has no valid timing).  Times
    are the exploration's single-replay ones (the first evaluation of a code object);
    a variant maps to the code object of its latest compile record."""
    from . import passes
    pool = pool if pool is not None else passes.load_pool()
    sample = space.sample_variants(family, pool, samples, seed)[:n]
    comp = {}
    for r in db.where(kind="compile", family=family):
        if r.get("status") == "ok":
            comp[r["key"]] = r["sha"]
        else:
            comp.pop(r["key"], None)
    times, base = {}, None
    for r in db.where(kind="eval", family=family, status="ok"):
        t = r.get("times", {}).get(str(size))
        if t:
            if r["sha"] == "default" and base is None:
                base = t
            times.setdefault(r["sha"], t)
    if not base:
        return []
    return [base / times[comp[v.key()]] if comp.get(v.key()) in times else None for v in sample]


def first100(db, family, size, samples=500, seed=5500, pool=None, n=100):
    """Speedups over the default of the first `n` sampled variants at `size` (those that
    compiled and ran correctly), in sample order."""
    return [x for x in _sample_speedups(db, family, size, samples, seed, pool, n) if x is not None]


def best_so_far(db, family, size, counts=(10, 50, 100, 200, 500), samples=500, seed=5500, pool=None):
    """Best speedup over the default at `size` among the first k sampled variants (failed
    ones included in k), for each k in `counts`: how the exploration converges with its
    sample size."""
    sp = _sample_speedups(db, family, size, samples, seed, pool, max(counts))
    out, best = {}, 0.0
    for i, x in enumerate(sp, 1):
        if x is not None:
            best = max(best, x)
        if i in counts:
            out[i] = best
    return out


def summarize_first100(sp):
    if not sp:
        return None
    return dict(n=len(sp), faster=sum(s > 1.02 for s in sp), same=sum(0.98 <= s <= 1.02 for s in sp),
                slower=sum(s < 0.98 for s in sp), half_or_worse=sum(s <= 0.5 for s in sp),
                best=max(sp), median=statistics.median(sp), worst=min(sp))
