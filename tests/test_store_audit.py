"""The gfx950 wide-store check (paper_1206_3215_amd/store_audit.py): its scan
on hand-written disassembly, and the built library's device code."""
import glob
import os

import pytest

from paper_1206_3215_amd import build, store_audit

HEAD = "0000000000001000 <k>:"


def scan(*body):
    return store_audit.audit_disassembly([HEAD, *body])


def test_overwrite_right_behind_a_wide_store_is_reported():
    bad = scan("buffer_store_dwordx4 v[22:25], v164, s[40:43], s75 offen",
               "v_fma_f64 v[22:23], -s[48:49], v[116:117], v[22:23]")
    assert len(bad) == 1 and bad[0][0] == "k" and bad[0][3] == 0


def test_global_store_data_operand_is_the_second():
    assert scan("global_store_dwordx4 v[4:5], v[0:3], off", "v_mul_f32_e32 v0, s5, v10")
    assert not scan("global_store_dwordx4 v[4:5], v[0:3], off", "v_mul_f32_e32 v4, s5, v10")


def test_two_wait_states_are_enough_and_nop_counts_its_length():
    assert not scan("buffer_store_dwordx4 v[2:5], v1, s[4:7], s0 offen", "s_nop 1", "v_add_f32_e32 v2, v6, v6")
    assert not scan("buffer_store_dwordx4 v[2:5], v1, s[4:7], s0 offen", "v_mov_b32_e32 v9, 0",
                    "s_mov_b32 s3, 0", "v_add_f32_e32 v2, v6, v6")
    assert scan("buffer_store_dwordx4 v[2:5], v1, s[4:7], s0 offen", "s_nop 0", "v_add_f32_e32 v2, v6, v6")


def test_narrow_stores_comparisons_and_other_registers_pass():
    assert not scan("buffer_store_dwordx2 v[2:3], v1, s[4:7], 0 offen", "v_mov_b32_e32 v2, 0")
    assert not scan("buffer_store_dwordx4 v[2:5], v1, s[4:7], 0 offen", "v_cmp_gt_u32_e32 vcc, s15, v2")
    assert not scan("buffer_store_dwordx4 v[2:5], v1, s[4:7], 0 offen", "v_mov_b32_e32 v6, 0")
    # a load into the store's registers is a write as well
    assert scan("buffer_store_dwordx4 v[2:5], v1, s[4:7], 0 offen", "ds_read_b64 v[4:5], v0")


def test_built_library_is_clean():
    objs = sorted(glob.glob(os.path.join(build.BUILD, "*.hip.o")))
    if not objs:
        pytest.skip("library not built (python -m paper_1206_3215_amd.build)")
    assert store_audit.audit(objs) == []
