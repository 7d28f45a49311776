"""Benchmark: 2D NLS split-step at 4096^2 (complex64) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the headline NLS configuration -- a 4096^2 periodic grid on
[-5pi,5pi)^2, psi0 = 0.5 exp(-r^2) (1 + 0.01 xi) with seeded noise xi,
dt = 1e-3, g = +1, FP32 complex fields.  A step is one Strang step (one row
pass and one column pass over the field).  K steps run in one nls_step call
between two device synchronisations; the field is resident in HBM before the
timed region starts.

Prints one JSON line with the throughput in grid-point-steps/s, a roofline
entry for the dominant kernel (its average launch duration measured with HIP
events on the plan's stream during a second timed run), and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
BYTES_PER_PT_PASS = {0: 16, 1: 32}  # read + write of one complex value, FP32 / FP64


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("fft_line.hpp", "kernels.hpp", "k_nls.hip", "pst_common.hpp"):
        with open(os.path.join(ROOT, "paper_1206_3215_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str, n_pts: int):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "nls_4096_fp32_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(n: int, dt: float, budget_s: float = 15.0):
    """The FP64 oracle (scipy FFT on all host cores) on the same grid and
    initial condition, for as many steps as fit in about budget_s."""
    from oracle import nls as onls
    from oracle import spectral as sp
    from paper_1206_3215_amd import inputs
    d = inputs.PAPER_DOMAIN
    psi = inputs.nls_gaussian(n, n, d, seed=0)
    t0 = time.perf_counter()
    psi = onls.step(psi, d.lx, d.ly, dt, 1.0)
    one = time.perf_counter() - t0
    steps = max(1, min(60, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(steps):
        psi = onls.step(psi, d.lx, d.ly, dt, 1.0)
    el = time.perf_counter() - t0
    return {"value": n * n * steps / el, "unit": "grid-pt-steps/s", "cores": sp.WORKERS,
            "kind": "oracle",
            "sample": f"NLS {n}^2 complex128 split-step, {steps} steps of dt={dt} "
                      f"(scipy.fft, {sp.WORKERS} workers), loop only"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(simulations are independent, see the sharding notes in the design document)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1206_3215_amd import binding as b
    from paper_1206_3215_amd import inputs

    torch.cuda.set_device(0)
    n, K, W = args.n, args.steps, args.warmup
    prec = b.PST_FP32 if args.prec == "fp32" else b.PST_FP64
    d = inputs.PAPER_DOMAIN
    dt, g = 1e-3, 1.0
    plan = b.Plan(n, n, b.PST_C2C, prec, 1)
    psi = torch.from_numpy(inputs.nls_gaussian(n, n, d, seed=0)).to("cuda", plan.complex_dtype)
    psi = psi.reshape(1, n, n).contiguous()
    q0 = plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g)

    # warmup
    if W > 0:
        plan.nls_step(psi, d, dt, g, W)
    torch.cuda.synchronize()

    # timed region: K steps
    t0 = time.perf_counter()
    plan.nls_step(psi, d, dt, g, K)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    q1 = plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g)
    value = n * n * K / el

    # second timed region with per-pass events -> dominant kernel's duration
    plan.profile_enable(True)
    plan.nls_step(psi, d, dt, g, K)
    torch.cuda.synchronize()
    row_ms, row_n = plan.profile_read(b.PASS_NLS_ROW)
    col_ms, col_n = plan.profile_read(b.PASS_NLS_COL)
    plan.profile_enable(False)
    passes = {"nls_row": (row_ms, row_n), "nls_col": (col_ms, col_n)}
    dom = max(passes, key=lambda k: passes[k][0])
    avg_s = passes[dom][0] / passes[dom][1] / 1e3
    alg_bytes = BYTES_PER_PT_PASS[prec] * n * n
    achieved = alg_bytes / avg_s / 1e9
    kname = {"nls_row": "k_nls_row", "nls_col": "k_nls_col"}[dom]
    traffic = traffic_from_profile(kname, n * n)

    # device-to-device copy bandwidth of the same field size, for context
    src = torch.empty(2 * alg_bytes // 2, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        dst.copy_(src)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 20 / (time.perf_counter() - t1) / 1e9

    out = {
        "metric": "grid-pt-steps/s & %HBM roofline, 2D NLS 4096^2",
        "value": value,
        "unit": "grid-pt-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == b.PST_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"nls_split_step_{n}x{n}_{args.prec}", "grid": [n, n],
                   "domain": "[-5pi,5pi)^2", "dt": dt, "g": g, "ic": "0.5exp(-r^2)(1+0.01xi), seed 0"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
                     "avg_launch_us": avg_s * 1e6, "bytes_per_launch_alg": alg_bytes},
        "pct_hbm_roofline_step": value * 2 * BYTES_PER_PT_PASS[prec] / (HBM_PEAK_GBS * 1e9),
        "passes_avg_us": {k: (v[0] / max(v[1], 1)) * 1e3 for k, v in passes.items()},
        "copy_GBps": copy_gbs,
        "mass_rel_drift": float(q1[0, 0] / q0[0, 0] - 1),
        "energy_rel_drift": float(q1[0, 1] / q0[0, 1] - 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
