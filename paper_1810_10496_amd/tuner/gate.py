"""Static check of a built code object before it may run on the GPU.

Random phase orders (Sec. 3: any pass, any position, repetition allowed) can
leave the device IR in shapes the standard pipelines never hand to the AMDGPU
back end, and the back end does not compile all of them correctly.  The one
known case: a stack object addressed through a generic (flat) pointer with a
negative constant offset.  Its flat address is the private aperture base plus
the object's frame offset plus the offset, a 64-bit sum that the back end
splits into a low add and a high add-with-carry; it folds the frame offset and
the constant into the low add's immediate (e.g. 0x60 + -4 -> 0x5c) and so drops
the carry that the high half (which still adds the constant's sign extension,
-1) relied on.  The pointer comes out 4 GiB below the aperture, and the first
access through it stops the queue with a memory-aperture violation.  Standard
pipelines run SROA and address-space inference, so their kernels never form
flat addresses of stack objects at all (`tests/data/aperture_carry.ll` is a
25-line kernel that shows the dropped carry with the installed `llc`; the same
kernel with the array in LDS instead of on the stack keeps the carry, and the
default FP32 rank-k kernel forms flat LDS addresses under -O3).

The gate rejects every code object that reads the private aperture base
(`src_private_base`): that is the only way a kernel forms a flat address of a
stack object, so the miscompiled arithmetic cannot reach the GPU.  It also
rejects kernels with a dynamically sized stack or a private segment beyond
`PRIVATE_LIMIT`, and group segments beyond the LDS of one CU.  The kernels of
this library, built with any standard pipeline, pass (checked by the CPU tests
for every family).
"""
from __future__ import annotations

import os
import re
import subprocess
import tempfile

from .. import codegen

APERTURE_REGS = ("src_private_base",)
PRIVATE_LIMIT = 4096            # bytes of private segment per work-item
GROUP_LIMIT = 160 * 1024        # LDS of one CU (gfx950)


def _tool(name):
    return codegen.tool(name)


def kernel_records(path: str) -> list[dict]:
    """Per-kernel records (name, segment sizes, stack) from the code object's metadata note."""
    import yaml
    r = subprocess.run([_tool("llvm-readelf"), "--notes", path], capture_output=True, text=True, timeout=60)
    if r.returncode != 0:
        raise RuntimeError(f"llvm-readelf failed: {r.stderr[-300:]}")
    m = re.search(r"^\s*---\s*$(.*?)^\.\.\.\s*$", r.stdout, re.S | re.M)
    if not m:
        raise RuntimeError("no AMDGPU metadata note")
    doc = yaml.safe_load(m.group(1)) or {}
    return [{k.lstrip("."): v for k, v in kern.items() if k != ".args"} for kern in doc.get("amdhsa.kernels", [])]


def disassembly(path: str) -> str:
    r = subprocess.run([_tool("llvm-objdump"), "-d", f"--mcpu={codegen.ARCH}", path], capture_output=True,
                       text=True, timeout=120)
    if r.returncode != 0:
        raise RuntimeError(f"llvm-objdump failed: {r.stderr[-300:]}")
    return r.stdout


def check_file(path: str) -> str | None:
    """None if the code object may run; otherwise the reason it may not."""
    text = disassembly(path)
    func, bad = "?", []
    for line in text.splitlines():
        m = re.match(r"^[0-9a-f]+ <([^>]+)>:", line)
        if m:
            func = m.group(1)
            continue
        if any(reg in line for reg in APERTURE_REGS) and func not in bad:
            bad.append(func)
    if bad:
        return f"flat addresses of stack objects (src_private_base) in {', '.join(bad)}"
    for rec in kernel_records(path):
        name = rec.get("name", "?")
        if rec.get("uses_dynamic_stack", False):
            return f"{name}: dynamically sized stack"
        if int(rec.get("private_segment_fixed_size", 0)) > PRIVATE_LIMIT:
            return f"{name}: private segment {rec['private_segment_fixed_size']} B > {PRIVATE_LIMIT}"
        if int(rec.get("group_segment_fixed_size", 0)) > GROUP_LIMIT:
            return f"{name}: group segment {rec['group_segment_fixed_size']} B > {GROUP_LIMIT}"
    return None


def check(code: bytes) -> str | None:
    """`check_file` for code object bytes."""
    fd, p = tempfile.mkstemp(suffix=".co", prefix="pkgate_")
    try:
        with os.fdopen(fd, "wb") as f:
            f.write(code)
        return check_file(p)
    finally:
        os.unlink(p)
