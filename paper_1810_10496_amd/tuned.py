"""The table of tuned variants: which code object to use per (family, size bucket).

The table is plain JSON (``tuned/best.json``), written by the tuner and read
here.  Each entry names a family, a size bucket (pk_size_bucket of the
problem's largest dimension), the knob values and the pass pipeline of the
chosen variant, and the SHA-256 of the code object the tuner measured.  Code
objects are rebuilt from that description (and cached under ``_build/tuned``);
an entry whose rebuilt code object does not hash to the recorded value is
rejected, so a table is only ever applied to the code it was measured with.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os

from . import codegen

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned", "best.json")
CACHE = os.path.join(HERE, "_build", "tuned")


def read_table(path: str = TABLE) -> list[dict]:
    if not os.path.exists(path):
        return []
    with open(path) as f:
        doc = json.load(f)
    return list(doc.get("entries", []))


def read_reuse(path: str = TABLE) -> list[dict]:
    """Feature-based reuse assignments: per (family, size, K) the carried-over variant."""
    if not os.path.exists(path):
        return []
    with open(path) as f:
        doc = json.load(f)
    return list(doc.get("reuse", []))


ORDERS = os.path.join(HERE, "tuned", "orders.json")


def read_orders(path: str = ORDERS) -> list[dict]:
    """The phase-order exploration's minimal best order per family (fixed default knobs),
    as entries like the table's (family, size, knobs, pipeline, code_sha256)."""
    if not os.path.exists(path):
        return []
    with open(path) as f:
        doc = json.load(f)
    out = []
    for fam, e in sorted(doc.get("families", {}).items()):
        if e.get("order") and e.get("code_sha256"):
            out.append(dict(family=fam, size=int(e["size"]), knobs=dict(codegen.FAMILIES[fam].defaults),
                            pipeline=",".join(e["order"]), llc_flags=["-O3"], opt_flags=[],
                            code_sha256=e["code_sha256"]))
    return out


def reuse_summary(path: str = TABLE) -> dict:
    """The tuner's own estimates (cosine K=1/3, random-K control) stored with the table."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        doc = json.load(f)
    return {k: v for k, v in doc.get("reuse_summary", {}).items() if k != "nearest"}


def _cache_path(e):
    return os.path.join(CACHE, f"{e['family']}_{e['code_sha256'][:16]}.co")


def code_for(entry: dict, build_missing: bool = True) -> bytes | None:
    p = _cache_path(entry)
    if os.path.exists(p):
        code = open(p, "rb").read()
        if hashlib.sha256(code).hexdigest() == entry["code_sha256"]:
            return code
    if not build_missing:
        return None
    b = codegen.compile_variant(entry["family"], entry.get("knobs", {}), entry.get("pipeline", codegen.DEFAULT_PIPELINE),
                                tuple(entry.get("llc_flags", ["-O3"])), opt_flags=tuple(entry.get("opt_flags", [])))
    if b.code_hash != entry["code_sha256"]:
        return None
    os.makedirs(CACHE, exist_ok=True)
    with open(p, "wb") as f:
        f.write(b.code)
    return b.code


def rebuild(entry: dict) -> bytes | None:
    """Compile an entry from its description now; the cache keeps the result only if it
    reproduces the recorded code object (a changed kernel source or tool chain makes
    the entry stale, and a stale cached copy is removed, never loaded)."""
    p = _cache_path(entry)
    try:
        b = codegen.compile_variant(entry["family"], entry.get("knobs", {}),
                                    entry.get("pipeline", codegen.DEFAULT_PIPELINE),
                                    tuple(entry.get("llc_flags", ["-O3"])),
                                    opt_flags=tuple(entry.get("opt_flags", [])))
    except codegen.CompileError:
        b = None
    if b is None or b.code_hash != entry["code_sha256"]:
        if os.path.exists(p):
            os.unlink(p)
        return None
    os.makedirs(CACHE, exist_ok=True)
    with open(p, "wb") as f:
        f.write(b.code)
    return b.code


def build_all(path: str = TABLE, jobs: int = 8) -> dict:
    """Rebuild every entry of the table from source into the cache; returns {sha: ok}."""
    entries = [e for e in read_table(path) + read_reuse(path) if not e.get("is_default")] + read_orders()
    uniq = list({e["code_sha256"]: e for e in entries}.values())
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(lambda e: rebuild(e) is not None, uniq))
    return {e["code_sha256"]: ok for e, ok in zip(uniq, res)}


def apply(ctx, path: str = TABLE, build_missing: bool = True) -> list[dict]:
    """Load the table's variants into `ctx` and register them as best per bucket.

    Returns the applied entries with their variant ids; entries whose code
    object cannot be reproduced are skipped (reported with ``vid = -1``)."""
    out = []
    for e in read_table(path):
        if e.get("is_default"):
            out.append(dict(e, vid=ctx.variant_default(e["family"])))
            continue
        code = code_for(e, build_missing)
        if code is None:
            out.append(dict(e, vid=-1))
            continue
        vid = ctx.variant_load(code)
        ctx.variant_set_best(e["family"], int(e["bucket"]), vid)
        out.append(dict(e, vid=vid))
    return out


def load_orders(ctx, path: str = ORDERS, build_missing: bool = True) -> dict:
    """Load each family's best phase order (not registered as best); {family: variant id}."""
    out = {}
    for e in read_orders(path):
        code = code_for(e, build_missing)
        if code is not None:
            out[e["family"]] = (ctx.variant_load(code), e)
    return out


def load_reuse(ctx, path: str = TABLE, build_missing: bool = True) -> dict:
    """Load the reuse assignments' code objects into `ctx` (not registered as best).

    Returns {(family, size, k): variant id}; default assignments map to the
    family's default variant, unreproducible ones are left out."""
    out, loaded = {}, {}
    for e in read_reuse(path):
        key = (e["family"], int(e["size"]), int(e["k"]))
        if e.get("is_default"):
            out[key] = ctx.variant_default(e["family"])
            continue
        sha = e["code_sha256"]
        if sha not in loaded:
            code = code_for(e, build_missing)
            loaded[sha] = ctx.variant_load(code) if code is not None else None
        if loaded[sha] is not None:
            out[key] = loaded[sha]
    return out
