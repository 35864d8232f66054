"""Command line of the tuner.

    python -m paper_1810_10496_amd.tuner passes                       # compile-level pass filter
    python -m paper_1810_10496_amd.tuner gpu-filter  --workdir D      # execution-level pass filter (GPU)
    python -m paper_1810_10496_amd.tuner explore     --workdir D [--families a,b] [--samples 500]
    python -m paper_1810_10496_amd.tuner finalize    --workdir D [--families a,b]
    python -m paper_1810_10496_amd.tuner refine      --workdir D [--families a,b] [--table path]
                                                                      # a structured grid into a finished table
    python -m paper_1810_10496_amd.tuner upgrade     --workdir D --families gemm_bf16_ws,gemm_split_ws
                                                                      # entries rebuilt with the EPI epilogue
    python -m paper_1810_10496_amd.tuner reuse       --workdir D
    python -m paper_1810_10496_amd.tuner table       --workdir D [--out path]
    python -m paper_1810_10496_amd.tuner report      --workdir D
    python -m paper_1810_10496_amd.tuner study       --workdir D --out study.md
    python -m paper_1810_10496_amd.tuner orders-<step> --workdir D ...  (random phase orders, tuner/orders.py)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys

from .. import codegen, workloads
from . import explore as X, passes, space


def log(*a):
    print(*a, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1810_10496_amd.tuner")
    ap.add_argument("cmd", choices=["passes", "gpu-filter", "explore", "finalize", "refine", "upgrade", "reuse", "table", "report",
                                        "study", "phase", "orders-build", "orders-eval", "orders-finalize",
                                        "orders-minimise", "orders-permute", "orders-cross", "orders-table",
                                        "orders-report", "table-report"])
    ap.add_argument("--workdir", default="tune_work")
    ap.add_argument("--families", default=",".join(workloads.TUNED_FAMILIES))
    ap.add_argument("--samples", type=int, default=500)
    ap.add_argument("--seed", type=int, default=5500)
    ap.add_argument("--sizes", default=",".join(map(str, workloads.SIZES)))
    ap.add_argument("--jobs", type=int, default=min(16, os.cpu_count() or 8))
    ap.add_argument("--max-minutes", type=float, default=None)
    ap.add_argument("--top", type=int, default=10)
    ap.add_argument("--out", default=None)
    ap.add_argument("--codir", default=None, help="directory for code objects (default <workdir>/co)")
    ap.add_argument("--table", default=None, help="phase: tuning table whose variants are minimised")
    ap.add_argument("--size", type=int, default=None, help="phase: the size timed (default: the largest)")
    ap.add_argument("--replays", type=int, default=10, help="phase: timed replays per variant")
    ap.add_argument("--build-only", action="store_true", help="phase: compile, do not evaluate")
    ap.add_argument("--only", action="append", default=[], metavar="KNOB=VALUE",
                    help="refine: keep only the grid settings with these knob values")
    ap.add_argument("--set", action="append", default=[], metavar="KNOB=VALUE",
                    help="upgrade: rebuild the families' entries with these knobs; an entry is "
                         "replaced only where that is faster by the margin")
    ap.add_argument("--stage", choices=["host", "gpu"], default="host",
                    help="orders-minimise/permute/cross: the host (compile) or the GPU (timing) half")
    a = ap.parse_args(argv)
    if a.codir:
        X.CODIR = a.codir
    fams = [f for f in a.families.split(",") if f]
    sizes = tuple(int(s) for s in a.sizes.split(","))

    if a.cmd == "passes":
        doc = passes.filter_pool(workloads.TUNED_FAMILIES, jobs=a.jobs, log=log)
        passes.save_pool(doc)
        return 0

    if a.cmd == "gpu-filter":
        from .evaluator import Evaluator
        doc = json.load(open(passes.POOL_FILE))
        pool = doc["pool"]
        db = X.DB(os.path.join(a.workdir, "db_filter.jsonl"))
        dropped = dict(doc.get("gpu_dropped", {}))
        for fam in fams:
            vs = [space.Variant(fam, space.default_knobs(fam), p) for p in pool]
            with cf.ThreadPoolExecutor(max_workers=a.jobs) as ex:
                built = list(ex.map(lambda v: X._build(v, a.workdir), vs))
            ev = Evaluator(fam, sizes, log=log, stderr_path=os.path.join(a.workdir, f"worker_{fam}.err"))
            for v, rec in zip(vs, built):
                db.add(dict(rec, kind="compile", filter=True))
                if rec["status"] != "ok":
                    dropped.setdefault(v.pipeline, f"{fam}: {rec['status']}")
                    continue
                res = ev.request(dict(op="eval", code=X._co_path(a.workdir, fam, rec["sha"]), validate=True,
                                      seeds=1, time=False), timeout=120)
                db.add(dict(kind="eval", family=fam, sha=rec["sha"], status=res.get("status"), filter=True,
                            detail=res.get("detail", "")))
                if res.get("status") != "ok":
                    dropped.setdefault(v.pipeline, f"{fam}: {res.get('status')} {res.get('detail', '')}"[:200])
                    log(f"[gpu-filter] {fam}: {v.pipeline} -> {res.get('status')}")
            ev.close()
            log(f"[gpu-filter] {fam} done; {len(dropped)} passes dropped so far")
        out = dict(doc, gpu_dropped=dropped)
        with open(os.path.join(a.workdir, "pass_pool.json"), "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
        return 0

    if a.cmd == "explore":
        pool = passes.load_pool(os.path.join(a.workdir, "pass_pool.json")) \
            if os.path.exists(os.path.join(a.workdir, "pass_pool.json")) else passes.load_pool()
        for fam in fams:
            c = X.explore(fam, a.workdir, a.samples, a.seed, sizes, a.jobs, log=log, max_minutes=a.max_minutes,
                          pool=pool)
            log(f"[explore] {fam} census: {json.dumps(c, sort_keys=True)}")
        return 0

    if a.cmd == "finalize":
        for fam in fams:
            ents = X.finalize(fam, a.workdir, sizes, top=a.top, log=log)
            for e in ents:
                log(f"[finalize] {fam}/{e['size']}: speedup {e['speedup']:.3f} "
                    f"({'default' if e['is_default'] else e['pipeline'][:40]})")
        return 0

    if a.cmd == "refine":
        from .. import tuned
        path = a.table or tuned.TABLE
        for fam in fams:
            if fam not in X.REFINE_GRIDS:
                continue
            only = dict((k, int(v)) for k, v in (o.split("=", 1) for o in a.only))
            grid = [g for g in X.REFINE_GRIDS[fam] if all(g.get(k) == v for k, v in only.items())]
            n = X.refine(fam, a.workdir, path, grid, sizes, log=log, tag="structured grid", jobs=a.jobs)
            log(f"[refine] {fam}: {n} entries replaced")
        return 0

    if a.cmd == "upgrade":
        # the prepared bf16 / split GEMM entries gain the prepared-operand epilogue (EPI),
        # which the chained product uses to write T straight into its second product
        from .. import tuned
        path = a.table or tuned.TABLE
        if a.set:
            extra = dict((k, int(v)) for k, v in (o.split("=", 1) for o in a.set))
            for fam in fams:
                if not all(k in space.REFINE_ONLY.get(fam, {}) or k in space.DOMAINS.get(fam, {}) for k in extra):
                    continue
                n = X.upgrade(fam, a.workdir, path, extra, sizes, log=log, tag=f"{extra} upgrade", jobs=a.jobs,
                              gain=True)
                log(f"[upgrade] {fam}: {n} entries upgraded")
            return 0
        for fam in fams:
            if fam in ("gemm_bf16_ws", "gemm_split_ws"):
                n = X.upgrade(fam, a.workdir, path, dict(EPI=1), sizes, log=log, tag="EPI upgrade", jobs=a.jobs)
                log(f"[upgrade] {fam}: {n} entries upgraded")
        return 0

    if a.cmd == "reuse":
        out = X.reuse(fams, a.workdir, sizes, jobs=a.jobs, log=log)
        log(json.dumps({k: v for k, v in out.items() if k != "transfers"}, indent=1))
        return 0

    if a.cmd == "table":
        out = a.out or os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tuned",
                                    "best.json")
        doc = X.write_table(fams, a.workdir, out)
        log(f"[table] {len(doc['entries'])} entries -> {out}")
        return 0

    if a.cmd == "study":
        from .study import study
        text = study(a.workdir, fams)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        else:
            log(text)
        return 0
    if a.cmd == "phase":
        from . import phase
        from .. import tuned
        entries = tuned.read_table(a.table or tuned.TABLE)
        phase.run(fams, a.workdir, entries, a.size or max(sizes), replays=a.replays, jobs=a.jobs, log=log,
                  build_only=a.build_only)
        return 0
    if a.cmd.startswith("orders-"):
        from . import orders as O
        ofams = [f for f in a.families.split(",") if f] if a.families != ",".join(workloads.TUNED_FAMILIES) \
            else list(O.FAMILIES)
        if a.cmd == "orders-build":
            O.build(ofams, a.workdir, passes.load_pool(), a.samples, a.seed if a.seed != 5500 else O.ORDER_SEED,
                    jobs=a.jobs, log=log)
        elif a.cmd == "orders-eval":
            O.evaluate(ofams, a.workdir, jobs=a.jobs, log=log, max_minutes=a.max_minutes)
        elif a.cmd == "orders-finalize":
            O.finalize(ofams, a.workdir, log=log)
        elif a.cmd == "orders-minimise":
            if a.stage == "host":
                O.minimise_host(ofams, a.workdir, jobs=a.jobs, log=log)
            else:
                O.minimise_gpu(ofams, a.workdir, log=log)
        elif a.cmd == "orders-permute":
            O.permute_host(ofams, a.workdir, jobs=a.jobs, log=log) if a.stage == "host" \
                else O.permute_gpu(ofams, a.workdir, log=log, max_minutes=a.max_minutes)
        elif a.cmd == "orders-cross":
            O.cross_host(ofams, a.workdir, jobs=a.jobs, log=log) if a.stage == "host" \
                else O.cross_gpu(ofams, a.workdir, log=log)
        elif a.cmd == "orders-table":
            out = a.out or os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tuned",
                                        "orders.json")
            O.write_table(a.workdir, ofams, out)
            log(f"[orders] table -> {out}")
        elif a.cmd == "orders-report":
            text = O.report(a.workdir, ofams)
            if a.out:
                with open(a.out, "w") as f:
                    f.write(text)
            else:
                log(text)
        return 0
    if a.cmd == "table-report":
        from .. import tuned
        from .study import table_report
        out = a.out or os.path.join(os.path.dirname(tuned.TABLE), "table.md")
        with open(out, "w") as f:
            f.write(table_report(a.table or tuned.TABLE))
        log(f"[table-report] -> {out}")
        return 0

    if a.cmd == "report":
        db = X.DB(os.path.join(a.workdir, "db.jsonl"))
        rep = {fam: X.census(db, fam) for fam in fams}
        log(json.dumps(rep, indent=1, sort_keys=True))
        return 0
    return 1


if __name__ == "__main__":
    sys.exit(main())
