"""Variant code generation: kernel source + knob values + LLVM pass pipeline -> gfx950 code object.

This is the library's analogue of the paper's offline compilation flow
(Sec. 2.3, Fig. "compilationflow"): the kernel is lowered to LLVM IR by the
front end, the IR is optimised by ``opt`` with a chosen phase order, and the
result is lowered to a device binary that the host loads directly (there with
``clCreateProgramWithBinary``, here with ``hipModuleLoadData``):

    clang -x hip --cuda-device-only -emit-llvm -O3 -Xclang -disable-llvm-passes
        (front-end IR with O3 metadata but no optimisation applied)
    opt -passes=<pipeline>              (the phase order under study)
    llc -mcpu=gfx950 -filetype=obj      (AMDGPU back end)
    ld.lld -shared                      (-> code object)

The built-in default of every family is the same flow with the standard
``default<O3>`` pipeline and the family's default knobs.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import tempfile
import threading
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
KDIR = os.path.join(CSRC, "kernels")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LLVM_BIN = os.path.join(ROCM, "llvm", "bin")
ARCH = "gfx950"
# packed FP32 instructions are disabled in every build of these kernels
NO_PACKED_FP32_CLANG = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
NO_PACKED_FP32_LLC = ["-mattr=-packed-fp32-ops"]
DEFAULT_PIPELINE = "default<O3>"


@dataclass(frozen=True)
class FamilySpec:
    name: str
    fid: int
    src: str
    fixed: dict
    defaults: dict
    op: str                     # the operation it serves (pk_kernel name)
    prec: str = "fp32"


def _fs(name, fid, src, fixed, defaults, op, prec="fp32"):
    return FamilySpec(name, fid, src, dict(fixed), dict(defaults), op, prec)


FAMILIES = {f.name: f for f in [
    _fs("gemm_f32", 0, "gemm.hip", {"PREC": 0},
        dict(BM=128, BN=128, BK=16, WAVES_M=2, WAVES_N=2, VEC=4, UNROLL=1, USE_LDS=1, ORDER=3, MF=16, LDS_PAD=4, FC=0, IL=0,
             DK=0),
        "gemm"),
    _fs("gemm_bf16", 1, "gemm_lp.hip", {"PREC": 1},
        dict(BM=256, BN=128, BK=32, WAVES_M=4, WAVES_N=2, VEC=4, STAGES=2, ORDER=3), "gemm", "bf16"),
    _fs("gemm_split", 2, "gemm_lp.hip", {"PREC": 2},
        dict(BM=256, BN=128, BK=32, WAVES_M=4, WAVES_N=2, VEC=4, STAGES=2, ORDER=3), "gemm", "split"),
    _fs("gemv", 3, "gemv.hip", {"GEMV_KIND": 0},
        dict(ROWS=1, WAVES=4, VEC=4, UNROLL=4, USE_LDS=0, ORDER=0, NTL=0), "gemv"),
    _fs("gemv_t", 4, "gemv.hip", {"GEMV_KIND": 1},
        dict(ROWS=64, WAVES=4, VEC=4, UNROLL=16, ORDER=0, FUSE=0, NTL=0), "gemv_t"),
    _fs("gemv_pair", 5, "gemv.hip", {"GEMV_KIND": 2},
        dict(ROWS=64, WAVES=4, VEC=4, UNROLL=16, ORDER=0, FUSE=0, NTL=0), "gemv_pair"),
    _fs("conv2d", 6, "conv.hip", {"CONV_KIND": 2},
        dict(VEC=4, TX=64, TY=4, ROWS=8, UNROLL=1, USE_LDS=0, ORDER=0, NTL=0), "conv2d"),
    _fs("conv3d", 7, "conv.hip", {"CONV_KIND": 3},
        dict(VEC=4, TX=64, TY=4, ROWS=16, UNROLL=1, USE_LDS=0, ORDER=0, YR=4, PF=1, NTL=0), "conv3d"),
    _fs("colstats", 8, "colstats.hip", {},
        dict(VEC=4, WAVES=4, ROWS=64, ORDER=0, FUSE=0, NTL=0, MG=0), "colstats"),
    _fs("syrk_f32", 9, "syrk32.hip", {},
        dict(BT=64, BK=16, WAVES_M=2, WAVES_N=2, VEC=4, STAGES=2, ORDER=0, IL=0), "corr"),
    _fs("syrk_bf16", 10, "gemm_bf.hip", {"PREC": 1, "SYRK": 1},
        dict(BM=128, BN=128, BK=64, WAVES_M=4, WAVES_N=4, ORDER=2, LDS_PAD=8, PIPE=1, DSTAGES=2, SCHED=1),
        "corr", "bf16"),
    _fs("syrk_split", 11, "gemm_bf.hip", {"PREC": 2, "SYRK": 1},
        dict(BM=128, BN=128, BK=64, WAVES_M=4, WAVES_N=4, ORDER=2, LDS_PAD=8, PIPE=1, DSTAGES=2, SCHED=1),
        "corr", "split"),
    _fs("convert", 12, "convert.hip", {}, dict(VEC=4, NTHREADS=256), "convert"),
    _fs("rankk", 13, "rankk.hip", {}, dict(BT=64, BK=16, WAVES_M=2, WAVES_N=2, VEC=4, UNROLL=1), "syrk"),
    _fs("gesummv", 14, "gesummv.hip", {}, dict(ROWS=1, WAVES=4, VEC=4, UNROLL=4, NTL=0), "gesummv"),
    _fs("fdtd", 15, "fdtd.hip", {}, dict(VEC=4, TX=64, TY=4), "fdtd2d"),
    _fs("gemm_bf16_ws", 16, "gemm_bf.hip", {"PREC": 1},
        dict(BM=256, BN=256, BK=64, WAVES_M=4, WAVES_N=4, ORDER=3, LDS_PAD=8, PIPE=1, DSTAGES=2, SCHED=1, EPI=0),
        "gemm", "bf16"),
    _fs("gemm_split_ws", 17, "gemm_bf.hip", {"PREC": 2},
        dict(BM=256, BN=256, BK=32, WAVES_M=4, WAVES_N=4, ORDER=3, LDS_PAD=8, PIPE=1, DSTAGES=2, SCHED=0, EPI=0),
        "gemm", "split"),
    _fs("stream", 18, "stream.hip", {}, dict(NTHREADS=256, UNROLL=4), "stream"),
]}
FAMILY_BY_ID = {f.fid: f for f in FAMILIES.values()}


class CompileError(RuntimeError):
    def __init__(self, stage: str, msg: str):
        super().__init__(f"{stage}: {msg}")
        self.stage = stage


@dataclass
class Built:
    family: str
    knobs: dict
    pipeline: str
    code: bytes
    code_hash: str
    ir_path: str | None = None
    timings: dict = field(default_factory=dict)


def tool(name: str) -> str:
    p = os.path.join(LLVM_BIN, name)
    if not os.path.exists(p):
        raise FileNotFoundError(f"LLVM tool {name} not found under {LLVM_BIN}")
    return p


def macro_flags(spec: FamilySpec, knobs: dict) -> list[str]:
    vals = dict(spec.defaults)
    vals.update(knobs or {})
    unknown = set(vals) - set(spec.defaults)
    if unknown:
        raise ValueError(f"unknown knobs for {spec.name}: {sorted(unknown)}")
    flags = [f"-D{k}={int(v)}" for k, v in sorted(spec.fixed.items())]
    flags += [f"-D{k}={int(v)}" for k, v in sorted(vals.items())]
    return flags


def _run(stage, cmd, timeout, cwd=None):
    try:
        r = subprocess.run(cmd, capture_output=True, timeout=timeout, cwd=cwd)
    except subprocess.TimeoutExpired:
        raise CompileError(stage, f"timed out after {timeout}s")
    if r.returncode != 0:
        raise CompileError(stage, (r.stderr or b"").decode(errors="replace")[-2000:])
    return r


def emit_ir(spec: FamilySpec, knobs: dict, out_bc: str, timeout: float = 120.0) -> None:
    """Front end only: un-optimised device IR (with O3 metadata) for one knob setting.

    The source is compiled by relative name from the kernel directory and the
    HIP compilation-unit id is pinned, so the code object depends only on the
    source text, the knobs and the pipeline (not on where the tree lives)."""
    cmd = [tool("clang"), "-x", "hip", f"--offload-arch={ARCH}", "--cuda-device-only",
           "-emit-llvm", "-c", "-O3", "-Xclang", "-disable-llvm-passes", "-std=c++17",
           f"-cuid=pk_{spec.name}", *NO_PACKED_FP32_CLANG, "-I.", "-I..", *macro_flags(spec, knobs),
           spec.src, "-o", os.path.abspath(out_bc)]
    _run("frontend", cmd, timeout, cwd=KDIR)


_FRONTEND = {}                  # (family, knobs) -> un-optimised device IR (bitcode bytes)
_FRONTEND_LOCK = threading.Lock()


def frontend_ir(family: str, knobs: dict | None = None, timeout: float = 120.0) -> bytes:
    """The front end's output for one knob setting, computed once per process: the IR
    depends only on the source, the family's fixed macros and the knobs, so variants
    that differ only in their pipeline (a phase-order exploration) share it."""
    spec = FAMILIES[family]
    key = (family, tuple(sorted(macro_flags(spec, knobs or {}))))
    with _FRONTEND_LOCK:
        hit = _FRONTEND.get(key)
    if hit is not None:
        return hit
    wd = tempfile.mkdtemp(prefix="pkfe_")
    try:
        bc = os.path.join(wd, "in.bc")
        emit_ir(spec, knobs or {}, bc, timeout)
        with open(bc, "rb") as f:
            code = f.read()
    finally:
        shutil.rmtree(wd, ignore_errors=True)
    with _FRONTEND_LOCK:
        if len(_FRONTEND) > 256:
            _FRONTEND.clear()
        _FRONTEND[key] = code
    return code


def compile_variant(family: str, knobs: dict | None = None, pipeline: str = DEFAULT_PIPELINE,
                    llc_flags: tuple = ("-O3",), workdir: str | None = None,
                    timeout: float = 120.0, keep_ir: bool = False, opt_flags: tuple = ()) -> Built:
    """Build one variant; raises CompileError naming the failing stage."""
    import time
    spec = FAMILIES[family]
    knobs = dict(knobs or {})
    own = workdir is None
    wd = tempfile.mkdtemp(prefix="pkcg_") if own else workdir
    os.makedirs(wd, exist_ok=True)
    t = {}
    try:
        bc = os.path.join(wd, "in.bc")
        obc = os.path.join(wd, "opt.bc")
        obj = os.path.join(wd, "out.o")
        co = os.path.join(wd, "out.co")
        t0 = time.time()
        with open(bc, "wb") as f:
            f.write(frontend_ir(family, knobs, timeout))
        t["frontend"] = time.time() - t0
        t0 = time.time()
        _run("opt", [tool("opt"), "-mtriple=amdgcn-amd-amdhsa", f"-mcpu={ARCH}", *opt_flags,
                     f"-passes={pipeline}", bc, "-o", obc], timeout)
        if not os.path.exists(obc) or os.path.getsize(obc) == 0:
            raise CompileError("opt", "no optimised IR produced")
        t["opt"] = time.time() - t0
        t0 = time.time()
        _run("llc", [tool("llc"), "-mtriple=amdgcn-amd-amdhsa", f"-mcpu={ARCH}",
                     *NO_PACKED_FP32_LLC, *llc_flags, "-filetype=obj", obc, "-o", obj], timeout)
        _run("lld", [tool("ld.lld"), "-shared", obj, "-o", co], timeout)
        t["backend"] = time.time() - t0
        with open(co, "rb") as f:
            code = f.read()
        if len(code) < 64:
            raise CompileError("lld", "empty code object")
        h = hashlib.sha256(code).hexdigest()
        ir_path = None
        if keep_ir and not own:
            ir_path = bc
        return Built(family, knobs, pipeline, code, h, ir_path, t)
    finally:
        if own:
            shutil.rmtree(wd, ignore_errors=True)


def default_variants():
    """(family name, default knobs) for every family, in id order."""
    return [(s.name, dict(s.defaults)) for s in sorted(FAMILIES.values(), key=lambda s: s.fid)]
