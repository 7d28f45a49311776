"""bench.py's command line and host-side helpers (no GPU needed)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_unknown_extra_section_is_refused_before_any_work():
    r = run_bench("--extra", "sg,bogus")
    assert r.returncode == 2 and "bogus" in r.stderr and r.stdout == ""


def test_cpu_baseline_returns_its_state_for_the_parity_figure():
    import bench
    from oracle import nls as onls
    from paper_1206_3215_amd import inputs
    cb, psi, steps = bench.cpu_baseline(32, 1e-3, budget_s=0.2)
    assert cb["kind"] == "oracle" and cb["unit"] == "grid-pt-steps/s" and cb["value"] > 0
    assert cb["cores"] >= 1 and f"{steps - 1} steps" in cb["sample"]
    # psi is the oracle's field after `steps` steps from the headline initial field
    d = inputs.PAPER_DOMAIN
    ref = onls.run(inputs.nls_gaussian(32, 32, d, seed=0), d.lx, d.ly, 1e-3, 1.0, steps)[0]
    assert np.allclose(psi, ref, rtol=0, atol=1e-12)


def test_kernel_source_hash_covers_the_nls_sources():
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    # a variant that was not counted has no record; the counted ones carry bytes only while the
    # kernel sources hash matches the one recorded with them
    assert bench.traffic_from_profile("k_nls_col", 99, "nls_4096_fp64_traffic.json") is None
    assert bench.traffic_from_profile("k_nls_col", 0, "no_such_profile.json") is None
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", "nls_4096_fp64_traffic.json")))
    got = bench.traffic_from_profile("k_nls_col", 4, "nls_4096_fp64_traffic.json")
    if rec["source_hash"] == h:
        assert got == rec["kernels"]["k_nls_col"]["variants"]["4"]["bytes_per_launch"]
    else:
        assert got is None
