"""C-ABI library: loads, exports every entry point include/pst.h declares,
and rejects bad arguments on the host before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pst.h")
LIB = os.path.join(ROOT, "paper_1206_3215_amd", "libpst.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\*?\s+\**([a-z0-9_]+)\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["fft2d_plan", "fft2d_exec", "fft2d_destroy", "nls_step", "sg_start", "sg_step",
                     "ns_step", "conserved_quantities", "solve_batch", "pst_last_error",
                     "pst_sync_status", "pst_workspace_size", "pst_set_workspace"]:
        assert required in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libpst.so not built")
    return C.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_plan_rejects_bad_sizes_on_host(lib):
    from paper_1206_3215_amd import binding as b
    h = C.c_void_p()
    # sizes must be 2^a 3^b 5^c in [4, 8192]: 3 is too small, 14 and 21 have a factor 7
    for nx, ny, kind, prec, batch in [(3, 64, 0, 0, 1), (64, 14, 0, 0, 1), (21, 64, 0, 0, 1), (2, 2, 0, 0, 1),
                                      (16384, 64, 0, 0, 1), (8000 * 2, 64, 0, 0, 1), (64, 64, 7, 0, 1),
                                      (64, 64, 0, 5, 1), (64, 64, 0, 0, 0)]:
        st = b.lib.fft2d_plan(nx, ny, kind, prec, batch, None, C.byref(h))
        assert st == b.PST_ERR_INVALID, (nx, ny, kind, prec, batch)
        assert b.lib.pst_last_error().decode() != ""
    assert b.lib.fft2d_plan(64, 64, 0, 0, 1, None, None) == b.PST_ERR_INVALID


def test_entry_points_reject_null_plan(lib):
    from paper_1206_3215_amd import binding as b
    p = b.NlsParams(b.Domain(1, 1, 0, 0), 1e-3, 1.0)
    assert b.lib.nls_step(None, None, C.byref(p), 1) == b.PST_ERR_INVALID
    assert b.lib.fft2d_exec(None, None, None, -1) == b.PST_ERR_INVALID
    assert b.lib.fft2d_destroy(None) == b.PST_ERR_INVALID
    assert b.lib.solve_batch(None, -1, None) in (b.PST_ERR_INVALID, b.PST_ERR_UNSUPPORTED)
    assert b.lib.pst_version().decode().startswith("pst")


def test_column_variant_table_on_host(lib):
    # the compiled column tiles follow the rules stated in pst.h: variant 0
    # fills 1024 threads / 150 KB of LDS; single-field passes of 4096 and
    # more add the split / wide / radix-8 variants; anything else has variant
    # 1 = half of variant 0's width; unknown variants and sizes are rejected
    from paper_1206_3215_amd import binding as b
    assert b.column_variants(b.PST_FP32, 4096, True) == [(4, 16, 0, 16), (4, 32, 1, 16), (4, 16, 1, 16),
                                                         (8, 32, 1, 16), (4, 16, 1, 16)]
    assert b.column_variants(b.PST_FP32, 8192, True) == [(2, 16, 0, 16), (2, 32, 1, 16), (2, 16, 1, 16),
                                                         (4, 32, 1, 16), (2, 16, 1, 16)]
    assert b.column_variants(b.PST_FP32, 4096, False) == [(4, 16, 0, 16), (2, 16, 0, 16), (1, 16, 0, 16)]
    assert b.column_variants(b.PST_FP32, 1024, False) == [(16, 16, 0, 16), (8, 16, 0, 16), (4, 16, 0, 16),
                                                          (2, 16, 0, 16)]
    assert b.column_variants(b.PST_FP32, 256, False) == [(16, 16, 0, 16), (8, 16, 0, 16)]
    assert b.column_variants(b.PST_FP64, 4096, True) == [(2, 16, 0, 16), (1, 16, 0, 16), (2, 32, 1, 16),
                                                         (2, 16, 1, 16), (4, 16, 1, 16), (2, 8, 1, 8)]
    assert b.column_variants(b.PST_FP64, 8192, True) == [(1, 16, 0, 16), (1, 16, 0, 16), (1, 32, 1, 16),
                                                         (1, 16, 1, 16), (2, 16, 1, 16), (1, 8, 1, 8)]
    assert b.column_variants(b.PST_FP64, 2048, True) == [(4, 16, 0, 16), (2, 16, 0, 16)]
    assert b.column_variants(b.PST_FP32, 1024, True) == [(16, 16, 0, 16), (8, 16, 0, 16)]
    assert b.column_variants(b.PST_FP32, 16, True) == [(16, 16, 0, 16), (8, 16, 0, 16)]
    for prec in (b.PST_FP32, b.PST_FP64):
        for e in range(2, 14):
            n = 1 << e
            for single in (True, False):
                for w, vpt, split, radix in b.column_variants(prec, n, single):
                    r = min(n, vpt)
                    esz = (4 if split else 8) * (2 if prec == b.PST_FP64 else 1)
                    assert w * (n // r) <= 1024 and w * (n + n // 16) * esz <= 150 * 1024, (prec, n, w, vpt)
                    assert radix in (min(n, 16), 8) and vpt % radix == 0
    w = C.c_int()
    assert b.lib.pst_column_variant_info(b.PST_FP32, 4096, 9, 1, C.byref(w), C.byref(w), C.byref(w),
                                         C.byref(w)) == b.PST_ERR_INVALID
    assert b.lib.pst_column_variant_info(b.PST_FP32, 3000, 0, 1, C.byref(w), C.byref(w), C.byref(w),
                                         C.byref(w)) == b.PST_ERR_INVALID
    assert b.lib.pst_set_column_variant(None, 0) == b.PST_ERR_INVALID


def test_row_variant_table_on_host(lib):
    # NLS in-place row pass: one line per block from 4096 on (default, split,
    # radix 8 split, radix 8 complex), row pairs below (default P, P/2, 2P)
    from paper_1206_3215_amd import binding as b
    assert b.row_variants(b.PST_FP64, 4096) == [(0, 16, 0, 16), (0, 16, 1, 16), (0, 8, 1, 8), (0, 8, 0, 8)]
    assert b.row_variants(b.PST_FP32, 8192) == [(0, 32, 1, 16), (0, 16, 1, 16), (0, 8, 1, 8), (0, 8, 0, 8)]
    assert b.row_variants(b.PST_FP32, 1024) == [(2, 16, 0, 16), (1, 16, 0, 16), (4, 16, 0, 16)]
    assert b.row_variants(b.PST_FP64, 2048) == [(1, 16, 0, 16), (2, 16, 0, 16)]
    for prec in (b.PST_FP32, b.PST_FP64):
        for e in range(2, 14):
            n = 1 << e
            vs = b.row_variants(prec, n)
            assert len(vs) >= 1
            for pairs, vpt, split, radix in vs:
                threads = n // vpt * (2 * pairs if pairs else 1)
                assert threads <= 1024 and vpt % radix == 0, (prec, n, pairs, vpt)
    assert b.lib.pst_set_row_variant(None, 0) == b.PST_ERR_INVALID
