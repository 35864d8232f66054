"""Host-only checks of the C ABI library and the code generator (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1810_10496_amd import _lib, codegen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pk_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (pk_\w+)", out))
    assert set(names) <= exported
    # and the binding declares exactly those
    assert {s[0] for s in _lib.SIGNATURES} == set(names)


def test_status_strings_and_version():
    lib = _lib.load()
    assert lib.pk_abi_version() == 1
    assert lib.pk_status_string(0) == b"ok"
    assert lib.pk_status_string(2) == b"invalid shape"
    assert lib.pk_status_string(99) == b"unknown status"


def test_size_bucket():
    lib = _lib.load()
    assert [lib.pk_size_bucket(d) for d in (0, 1, 2, 3, 256, 257, 1000, 2048, 4096)] == \
        [0, 0, 1, 2, 8, 9, 10, 11, 12]


def ws(kernel, dims, prec=0):
    lib = _lib.load()
    arr = (ctypes.c_int64 * len(dims))(*dims)
    out = ctypes.c_size_t(123)
    st = lib.pk_workspace_bytes(kernel, arr, len(dims), prec, ctypes.byref(out))
    return st, out.value


def test_workspace_bounds():
    assert ws(0, [512, 512, 512]) == (0, 0)                           # gemm
    assert ws(1, [2048, 2048, 2048, 2048]) == (0, 2048 * 2048 * 4)   # gemm3: T
    a256 = lambda b: (b + 255) // 256 * 256                           # noqa: E731
    ld = lambda n: (n + 63) // 64 * 64                                # noqa: E731  partial row stride
    cell = 256                                                        # bytes per ticket cell
    # gemv_t: partials of the smallest row blocks (16 rows), then one ticket cell per
    # narrowest strip (64 columns)
    st, b = ws(3, [4096, 4096])
    assert st == 0 and b == a256((4096 // 16) * ld(4096) * 4) + (4096 // 64) * cell
    st, b2 = ws(4, [4096, 4096])                                      # pair: + row-block cells, y1 partials
    assert st == 0 and b2 == (a256((4096 // 16) * ld(4096) * 4) + (4096 // 64 + 4096 // 16) * cell
                              + (4096 // 64) * 4096 * 4)
    st, b = ws(3, [300, 70])
    assert st == 0 and b == a256(19 * 128 * 4) + 2 * cell
    st, b = ws(8, [2048, 2048])                                       # corr: colstats partials + cells
    assert st == 0 and b == a256((2048 // 16) * 3 * ld(2048) * 4) + (2048 // 64) * cell
    assert ws(3, [-1, 4])[0] == 2                                     # negative -> SHAPE
    assert ws(42, [1, 1])[0] == 1                                     # bad kernel -> INVALID_ARG
    assert ws(1, [1, 1])[0] == 1                                      # too few dims
    assert ws(0, [1, 1, 1], prec=7)[0] == 1                           # bad precision
    # pk_sgemm_ws: bf16 one plane, split two, of A [M][Kp] and B^T [N][Kp], Kp = K up to 64
    assert ws(0, [300, 200, 129], prec=1) == (0, a256(300 * 192 * 2) + a256(200 * 192 * 2))
    assert ws(0, [300, 200, 129], prec=2) == (0, 2 * (a256(300 * 192 * 2) + a256(200 * 192 * 2)))
    assert ws(0, [5, 6, 0], prec=1) == (0, a256(5 * 64 * 2) + a256(6 * 64 * 2))    # K = 0 still pads
    # gemm3 in bf16: T, then the larger of the two products' prepared operands
    M, N, K, L = 100, 37, 129, 65
    t = a256(M * L * 4)
    p1 = a256(M * 192 * 2) + a256(L * 192 * 2)
    p2 = a256(M * 128 * 2) + a256(N * 128 * 2)
    assert ws(1, [M, N, K, L], prec=1) == (0, t + max(p1, p2))
    # ... or, when the first product writes T straight into the second's prepared operand,
    # T's bf16 planes ([M][L up to 64]) and the larger of the first product's operands and
    # the second's C^T: whichever is larger (here L = 1, the direct layout)
    L = 1
    old = a256(M * L * 4) + max(a256(M * 192 * 2) + a256(L * 192 * 2), a256(M * 64 * 2) + a256(N * 64 * 2))
    direct = a256(M * 64 * 2) + max(a256(M * 192 * 2) + a256(L * 192 * 2), a256(N * 64 * 2))
    assert direct > old and ws(1, [M, N, K, L], prec=1) == (0, direct)
    direct2 = a256(2 * M * 64 * 2) + max(2 * (a256(M * 192 * 2) + a256(L * 192 * 2)), 2 * a256(N * 64 * 2))
    old2 = a256(M * L * 4) + 2 * max(a256(M * 192 * 2) + a256(L * 192 * 2), a256(M * 64 * 2) + a256(N * 64 * 2))
    assert ws(1, [M, N, K, L], prec=2) == (0, max(direct2, old2))
    # corr / covar in bf16 / split: + Z^T planes [m][n rounded up to 64]
    part = a256((130 // 16 + 1) * 3 * ld(70) * 4) + 2 * cell
    assert ws(8, [130, 70]) == (0, part)
    assert ws(8, [130, 70], prec=1) == (0, a256(part) + a256(70 * 192 * 2))
    assert ws(8, [130, 70], prec=2) == (0, a256(part) + 2 * a256(70 * 192 * 2))
    cov = a256(part) + 2 * a256(70 * 4)
    assert ws(10, [130, 70]) == (0, cov)
    assert ws(10, [130, 70], prec=2) == (0, cov + 2 * a256(70 * 192 * 2))


def test_null_context_is_rejected_without_touching_hip():
    lib = _lib.load()
    f = (ctypes.c_float * 9)()
    assert lib.pk_sgemm(None, 0, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, None) == 1
    assert lib.pk_conv2d_3x3(None, 4, 4, f, None, 4, None, 4, None) == 1
    assert b"context" in lib.pk_last_error()
    assert lib.pk_variant_select(None, 0, -1) == 1
    assert lib.pk_graph_launch(None, None) == 1


def test_context_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.pk_context_create(0, ctypes.byref(h))
    assert st != 0 and not h.value


def test_default_code_objects_carry_knob_records():
    manifest_dir = os.path.join(ROOT, "paper_1810_10496_amd", "_build")
    for spec in codegen.FAMILIES.values():
        co = os.path.join(manifest_dir, f"{spec.name}.co")
        assert os.path.exists(co), co
        syms = subprocess.run([codegen.tool("llvm-readelf"), "-s", co], capture_output=True,
                              text=True, check=True).stdout
        assert "pk_knobs" in syms
        names = _lib_fn_names(spec.fid)
        for n in names:
            assert re.search(rf"\b{n}\b", syms), (spec.name, n)


def _lib_fn_names(fid):
    table = {0: ["pk_gemm"], 1: ["pk_gemm"], 2: ["pk_gemm"], 3: ["pk_gemv"],
             4: ["pk_gemvt_partial", "pk_colsum_reduce"], 5: ["pk_gemv_pair_partial", "pk_colsum_reduce"],
             6: ["pk_conv2d"], 7: ["pk_conv3d"], 8: ["pk_colstats_partial", "pk_colstats_merge"],
             9: ["pk_syrk"], 10: ["pk_gemm_bf", "pk_corr_prep"], 11: ["pk_gemm_bf", "pk_corr_prep"],
             12: ["pk_convert", "pk_fill"],
             13: ["pk_rankk_syrk", "pk_rankk_syr2k"], 14: ["pk_gesummv", "pk_colsum_accumulate"],
             15: ["pk_fdtd_e", "pk_fdtd_h"], 16: ["pk_gemm_bf", "pk_gemm_prep"],
             17: ["pk_gemm_bf", "pk_gemm_prep"], 18: ["pk_stream_read", "pk_stream_copy"]}
    return table[fid]


def test_compile_variant_rejects_unknown_knob_and_bad_pipeline():
    with pytest.raises(ValueError):
        codegen.compile_variant("gemv", {"NOPE": 1})
    with pytest.raises(codegen.CompileError) as e:
        codegen.compile_variant("gemv", {}, pipeline="function(no-such-pass)")
    assert e.value.stage == "opt"


def test_knob_values_reach_the_code_object():
    b = codegen.compile_variant("gemv", {"ROWS": 2, "WAVES": 2, "VEC": 2})
    import tempfile
    p = tempfile.mktemp(suffix=".co")
    open(p, "wb").write(b.code)
    out = subprocess.run([codegen.tool("llvm-readelf"), "-x", ".rodata", p], capture_output=True,
                         text=True).stdout
    os.remove(p)
    # family 3 (gemv), TM=ROWS=2, TN=64*VEC=128 -> little-endian words 03000000 02000000 80000000
    flat = "".join(re.findall(r"0x[0-9a-f]+\s+((?:[0-9a-f]{8}\s+){1,4})", out)).replace(" ", "").replace("\n", "")
    assert "030000000200000080000000" in flat
