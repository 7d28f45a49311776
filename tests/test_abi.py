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
    for nx, ny, kind, prec, batch in [(3, 64, 0, 0, 1), (64, 12, 0, 0, 1), (2, 2, 0, 0, 1),
                                      (16384, 64, 0, 0, 1), (64, 64, 7, 0, 1), (64, 64, 0, 5, 1),
                                      (64, 64, 0, 0, 0)]:
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
