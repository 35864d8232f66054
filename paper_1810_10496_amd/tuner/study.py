"""The exploration study as a report: what the sampled variants did, where the
gains come from, and how well variants carry over between kernel families.

    python -m paper_1810_10496_amd.tuner study --workdir D --out study.md

Sections (all from the exploration DB, the finalized tables and reuse.json):
  census         per family: variants sampled, distinct code objects, outcome
                 categories (the paper's failure classes, Sec. 3.2)
  tuned vs default per family and size (finalist timings)
  attribution    best speedup over the default reachable by changing only the
                 pass pipeline (default knobs) and only the knobs (default
                 pipeline), from the exploration timings (Sec. 3.4 asks the same
                 question of its phase orders)
  pipelines      how the pipeline kinds are represented among each family's ten
                 fastest code objects at the largest size
  transfer       cross-family matrix: geomean over sizes of default / time of the
                 source family's best variant carried to the target (Sec. 4)
  reuse          cosine K = 1, 3 vs the random-K control (Sec. 4.2)
"""
from __future__ import annotations

import collections
import json
import math
import os

from .. import codegen
from . import explore as X, passes, space

SIZES = ("256", "512", "1000", "2048", "4096")


def _gm(xs):
    xs = [x for x in xs if x and x > 0]
    return math.exp(sum(math.log(x) for x in xs) / len(xs)) if xs else float("nan")


def _pipe_kind(v):
    if v["pipeline"] == codegen.DEFAULT_PIPELINE and not v.get("opt_flags") and \
            list(v.get("llc_flags", ["-O3"])) == ["-O3"]:
        return "default<O3>"
    if v.get("opt_flags") or list(v.get("llc_flags", ["-O3"])) != ["-O3"]:
        return "O3 + flags"
    return v["pipeline"]


def _sample(fam, samples, seed):
    pool = passes.load_pool()
    return [space.default_variant(fam)] + space.sample_variants(fam, pool, samples, seed)


def _phase_sections(db, workdir, families, samples, seed):
    from . import phase
    out = []
    pp = os.path.join(workdir, "phase.json")
    ph = json.load(open(pp)) if os.path.exists(pp) else {}
    lv_fams = [f for f in families if f in ph and ph[f].get("levels")]
    if lv_fams:
        levels = [lv for lv in space.STANDARD]
        out += ["", "## Standard levels at the default knobs (Sec. 3.1)", "",
                "Default knobs under each standard pipeline, time relative to default<O3> (above 1 = faster),",
                f"{ph[lv_fams[0]]['size']} elements per dimension (the 3D stencil: its 256^3 grid), 10 replays.", "",
                "| family | " + " | ".join(levels) + " |", "|---|" + "---:|" * len(levels)]
        for fam in lv_fams:
            t = ph[fam]["levels"]
            o3 = t.get("default<O3>")
            out.append(f"| {fam} | " + " | ".join(
                "-" if not (o3 and t.get(lv)) else f"{o3 / t[lv]:.3f}" for lv in levels) + " |")
    mi_fams = [f for f in families if f in ph and ph[f].get("minimise")]
    if mi_fams:
        out += ["", "## Minimising the tuned variants' flags (the Table 1 procedure)", "",
                "Each family's tuned variant at that size whose pipeline carries flags, re-timed as tuned, without",
                f"each flag, and without any; a flag stays in the minimal set when removing it costs more than "
                f"{phase.MARGIN:.0%}.", "",
                "| family | flags | tuned ms | flag-free ms | flag-free / tuned | minimal set |",
                "|---|---|---:|---:|---:|---|"]
        for fam in mi_fams:
            m = ph[fam]["minimise"]
            t, n = m.get("tuned"), m.get("without flags")
            out.append(f"| {fam} | {' '.join(ph[fam].get('flags', []))} | "
                       + ("-" if not t else f"{t:.4f}") + " | " + ("-" if not n else f"{n:.4f}") + " | "
                       + ("-" if not (t and n) else f"{n / t:.3f}")
                       + f" | {' '.join(ph[fam].get('minimal', [])) or '(none)'} |")
    rows = []
    for fam in families:
        big = max((int(s) for s in SIZES if any(s in r.get("times", {}) for r in db.where(
            kind="eval", family=fam, sha="default"))), default=None)
        if big is None:
            continue
        s = phase.summarize_first100(phase.first100(db, fam, big, samples, seed))
        if s:
            rows.append(f"| {fam} | {big} | {s['n']} | {s['faster']} | {s['same']} | {s['slower']} | "
                        f"{s['half_or_worse']} | {s['best']:.2f}x | {s['median']:.2f}x | {s['worst']:.2f}x |")
    if rows:
        out += ["", "## The first 100 sampled variants (Sec. 3.3)", "",
                "Speedup over the default at the largest size of the first 100 variants of the sample that",
                "compiled and ran correctly (faster / same / slower: beyond, within, below 2%).", "",
                "| family | size | n | faster | same | slower | at most 0.5x | best | median | worst |",
                "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"] + rows
    conv = []
    counts = (10, 50, 100, 200, 500)
    for fam in families:
        have = sorted({int(s) for s in SIZES if any(s in r.get("times", {}) for r in db.where(
            kind="eval", family=fam, sha="default"))})
        for size in sorted({s for s in have if s in (1000, max(have, default=0))}):
            b = phase.best_so_far(db, fam, size, counts, samples, seed)
            if b:
                conv.append(f"| {fam} | {size} | " + " | ".join(
                    "-" if k not in b else f"{b[k]:.2f}x" for k in counts) + " |")
    if conv:
        out += ["", "## Best speedup within the first k samples", "",
                "How the exploration converges with its sample size (the paper samples 10,000 orders per",
                "kernel): the best single-replay speedup over the default among the first k sampled variants,",
                "at 1000 (where tuning gains most) and at the largest size.",
                "", "| family | size | " + " | ".join(f"k={k}" for k in counts) + " |",
                "|---|---:|" + "---:|" * len(counts)] + conv
    out += ["", "The order of a standard pipeline's passes is fixed and flags have no order, so the paper's",
            "permutation experiment applies to the random phase orders: orders.md."]
    return out


def study(workdir, families, samples=500, seed=5500, note=None, explored=None):
    """`explored`: the families whose exploration rows the database holds (default: all);
    the census, attribution, pipeline and sample sections cover only those."""
    db = X.DB(os.path.join(workdir, "db.jsonl"))
    explored = list(families) if explored is None else [f for f in families if f in explored]
    keys = {fam: {v.key() for v in _sample(fam, samples, seed)} for fam in families}

    def sample_compiles(fam):
        """{sha: variant} of the current sample's successfully compiled variants"""
        return {r["sha"]: r["variant"] for r in db.where(kind="compile", family=fam, status="ok")
                if r["key"] in keys[fam]}
    out = ["# Variant exploration study", "",
           "Generated by `python -m paper_1810_10496_amd.tuner study` from the exploration database,",
           "the finalized per-size tables and the reuse evaluation.  Times are ms per launch.", ""]
    if note:
        out += [note, ""]
    # -- census
    out += ["## Census", "", "| family | variants | distinct code objects | outcomes |", "|---|---:|---:|---|"]
    for fam in explored:
        c = X.census(db, fam, keys[fam])
        rest = ", ".join(f"{k} {v}" for k, v in sorted(c.items()) if k not in ("variants", "distinct_code_objects"))
        out.append(f"| {fam} | {c.get('variants', 0)} | {c.get('distinct_code_objects', 0)} | {rest} |")
    # -- tuned vs default
    out += ["", "## Tuned vs default (finalists re-timed, 30 replays; 3% margin)", "",
            "| family | " + " | ".join(SIZES) + " |", "|---|" + "---:|" * len(SIZES)]
    for fam in families:
        p = os.path.join(workdir, f"table_{fam}.json")
        if not os.path.exists(p):
            continue
        t = {str(e["size"]): e for e in json.load(open(p))}
        cells = []
        for s in SIZES:
            e = t.get(s)
            cells.append("-" if e is None else (f"{e['speedup']:.2f}x" + ("" if not e["is_default"] else " (default)")))
        out.append(f"| {fam} | " + " | ".join(cells) + " |")
    # -- attribution
    out += ["", "## Where the gains come from (exploration timings)", "",
            "Best speedup over the default at each size among variants that differ from the default only",
            "in the pass pipeline and flags (knobs = default), only in the knobs (pipeline = default<O3>),",
            "and in both (- where the sample holds no variant of that kind; the phase-order section below",
            "times the default knobs under every standard level).", "",
            "| family | size | pipeline only | knobs only | both |", "|---|---:|---:|---:|---:|"]
    for fam in explored:
        dflt = codegen.FAMILIES[fam].defaults
        comp = sample_compiles(fam)
        evals = [r for r in db.where(kind="eval", family=fam, status="ok")]
        base = next((r["times"] for r in evals if r["sha"] == "default"), {})
        for s in SIZES:
            if s not in base:
                continue
            best = {"pipe": None, "knobs": None, "both": None}     # None: no such variant sampled
            for r in evals:
                v = comp.get(r["sha"])
                if v is None or s not in r.get("times", {}):
                    continue
                sp = base[s] / r["times"][s]
                same_k = all(v["knobs"].get(k) == dflt[k] for k in dflt if k in v["knobs"])
                same_p = _pipe_kind(v) == "default<O3>"
                key = "pipe" if same_k and not same_p else ("knobs" if same_p and not same_k else "both")
                best[key] = sp if best[key] is None else max(best[key], sp)
            cell = lambda x: "-" if x is None else f"{x:.2f}x"
            out.append(f"| {fam} | {s} | {cell(best['pipe'])} | {cell(best['knobs'])} | {cell(best['both'])} |")
    # -- pipelines among the fastest
    out += ["", "## Pipelines among each family's ten fastest code objects (largest size)", "",
            "| family | pipeline kinds |", "|---|---|"]
    for fam in explored:
        comp = sample_compiles(fam)
        evals = [r for r in db.where(kind="eval", family=fam, status="ok") if r["sha"] in comp]
        big = max((s for s in SIZES if any(s in r.get("times", {}) for r in evals)), key=int, default=None)
        if big is None:
            continue
        top = sorted((r for r in evals if big in r.get("times", {})), key=lambda r: r["times"][big])[:10]
        cnt = collections.Counter(_pipe_kind(comp[r["sha"]]) for r in top)
        out.append(f"| {fam} | " + ", ".join(f"{k} {v}" for k, v in cnt.most_common()) + " |")
    # -- phase-order analysis (levels, flag minimisation, first 100 samples)
    out += _phase_sections(db, workdir, explored, samples, seed)
    # -- transfer matrix and reuse
    rp = os.path.join(workdir, "reuse.json")
    if os.path.exists(rp):
        r = json.load(open(rp))
        tables = {}
        for fam in families:
            p = os.path.join(workdir, f"table_{fam}.json")
            if os.path.exists(p):
                tables[fam] = {str(e["size"]): e["default_ms"] for e in json.load(open(p))}
        fams = [f for f in families if f in tables and any(k.startswith(f + "<-") for k in r["transfers"])]
        out += ["", "## Transfer matrix", "",
                "Row = target family, column = source family: geomean over sizes of default time / time of the",
                "source's best variant carried over (knobs the two share, the source's pipeline); 1.00 = no",
                "change, blank = same family.", "",
                "| target \\ source | " + " | ".join(fams) + " |", "|---|" + "---:|" * len(fams)]
        for t in fams:
            cells = []
            for src in fams:
                if src == t:
                    cells.append("")
                    continue
                sp = []
                for s in SIZES:
                    v = r["transfers"].get(f"{t}<-{src}@{s}")
                    if v and s in tables[t]:
                        sp.append(tables[t][s] / v)
                cells.append(f"{_gm(sp):.2f}" if sp else "-")
            out.append(f"| {t} | " + " | ".join(cells) + " |")
        out += ["", "## Reuse (Sec. 4.2)", "",
                f"- nearest by cosine distance: " + "; ".join(f"{k}: {', '.join(v)}" for k, v in r["nearest"].items()),
                f"- geomean speedup over all (family, size): tuned {r['tuned']:.3f}x, cosine K=1 "
                f"{r['cosine_k1']:.3f}x, K=3 {r['cosine_k3']:.3f}x; random K=1 {r['random_k1']:.3f}x, "
                f"K=3 {r['random_k3']:.3f}x (1000 draws)"]
    return "\n".join(out) + "\n"


def table_report(table_path) -> str:
    """The finished tuning table as a report: per family and size the tuned / default
    speedup the table records and the step that chose the entry (the seeded exploration's
    finalize, a structured or one-launch `refine` grid, or an `upgrade`), and the entry's
    knobs where a later step changed them.  Written from the table alone."""
    with open(table_path) as f:
        doc = json.load(f)
    ents = doc["entries"]
    fams = sorted({e["family"] for e in ents})
    sizes = sorted({int(e["size"]) for e in ents})
    by = {(e["family"], int(e["size"])): e for e in ents}

    def step(e):
        if e.get("is_default"):
            return "default kept"
        src = e.get("source")
        return src if src else "finalize"

    out = ["# The tuning table (tuned/best.json)", "",
           "Speedup of the selected variant over the family's default at each size, as the step "
           "that selected it measured it (finalize: the seeded exploration's finalists, 30 "
           "replays; refine and upgrade: 30 replays beside the entry they replaced, which they "
           "beat by the 3% margin or, for a capability, matched within it).  Written by "
           "`python -m paper_1810_10496_amd.tuner table-report`.", "",
           "| family | " + " | ".join(str(s) for s in sizes) + " |",
           "|---|" + "---:|" * len(sizes)]
    for fam in fams:
        cells = []
        for s in sizes:
            e = by.get((fam, s))
            cells.append("—" if e is None else ("1.00x (default)" if e.get("is_default")
                                               else f"{float(e['speedup']):.2f}x"))
        out.append(f"| {fam} | " + " | ".join(cells) + " |")
    counts = collections.Counter(step(e) for e in ents)
    out += ["", "## Which step selected each entry", "",
            "| step | entries |", "|---|---:|"]
    out += [f"| {k} | {counts[k]} |" for k in sorted(counts)]
    later = [e for e in ents if e.get("source")]
    if later:
        out += ["", "## Entries selected after the exploration", "",
                "| family | size | step | tuned ms | speedup | knobs |", "|---|---:|---|---:|---:|---|"]
        for e in sorted(later, key=lambda e: (e["family"], int(e["size"]))):
            ks = ", ".join(f"{k}={v}" for k, v in sorted(e["knobs"].items()))
            out.append(f"| {e['family']} | {e['size']} | {e['source']} | {float(e['tuned_ms']):.4f} | "
                       f"{float(e['speedup']):.2f}x | {ks} |")
    return "\n".join(out) + "\n"
