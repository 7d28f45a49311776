"""Benchmark: 2D NLS split-step at 4096^2 (complex64) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32|fp64] [--no-cpu-baseline]
                    [--serve COUNT] [--extra [sg,ns,nls]] [--sweep]

Workload: the headline NLS configuration -- a 4096^2 periodic grid on
[-5pi,5pi)^2, psi0 = 0.5 exp(-r^2) (1 + 0.01 xi) with seeded noise xi,
dt = 1e-3, g = +1, FP32 complex fields.  A step is one Strang step (one row
pass and one column pass over the field).  K steps run in one nls_step call
between two device synchronisations; the field is resident in HBM before the
timed region starts.

Prints one JSON line with the throughput in grid-point-steps/s, a roofline
entry for the dominant kernel (its average launch duration measured with HIP
events on the plan's stream during a second timed run), the serving mix's
p50/p99 latency against the plain one-request-at-a-time path, and the FP64
CPU oracle timed on a bounded sample of the same workload together with the
device field's deviation from it after the same steps.  Progress lines for
finished sections go to stderr.
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


def traffic_from_profile(kernel: str, column_variant: int):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources and (for the column pass) the same
    column variant."""
    path = os.path.join(ROOT, "profiles", "nls_4096_fp32_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None or k.get("column_variant", column_variant) != column_variant:
        return None
    return k.get("bytes_per_launch")


def progress(msg: str) -> None:
    """One line per finished section on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
                      f"(scipy.fft, {sp.WORKERS} workers), loop only"}, psi, steps + 1


def bench_serve(count: int):
    """Serving mix: Poisson arrivals, equation uniform over {NLS, SG, NS},
    n = 2^e with e uniform on 7..11, steps uniform on 100..2000, FP32.
    The arrival rate is set to 0.8x the batched capacity measured on the same
    mix served all at once; p50/p99 latency and throughput are then measured
    with real-time arrivals, and the plain one-at-a-time path is timed on the
    same requests."""
    import torch

    from paper_1206_3215_amd import inputs
    from paper_1206_3215_amd.serve import GpuExecutor, Server, fifo_baseline
    budget = 16 << 30
    mix0 = inputs.serving_mix(count, rate_hz=1.0)
    work = sum(r.n * r.n * r.steps for r in mix0)
    ex = GpuExecutor()
    cap = Server(ex, budget, chunk=64).run(mix0, realtime=False).summary()
    rate = 0.8 * cap["pt_steps_per_s"] / (work / count)
    mix = inputs.serving_mix(count, rate_hz=rate)
    rep = Server(ex, budget, chunk=64).run(mix, realtime=True).summary()
    fifo_wall, fifo_rate, _ = fifo_baseline(mix)
    torch.cuda.synchronize()
    return {"requests": count, "hbm_budget_GiB": budget / 2 ** 30, "arrival_rate_hz": rate,
            "batched_capacity_pt_steps_per_s": cap["pt_steps_per_s"],
            "pt_steps_per_s": rep["pt_steps_per_s"], "p50_latency_s": rep["p50_latency_s"],
            "p99_latency_s": rep["p99_latency_s"], "wall_s": rep["wall_s"],
            "fifo_pt_steps_per_s": fifo_rate, "fifo_wall_s": fifo_wall,
            "batched_over_fifo": cap["pt_steps_per_s"] / fifo_rate}


def bench_sg(b, inputs):
    """Sine-Gordon 2048^2 FP32, 16 seeds in one launch, 500 steps of dt 0.01."""
    import torch
    n, B, dt, steps = 2048, 16, 0.01, 500
    d = inputs.PAPER_DOMAIN
    plan = b.Plan(n, n, b.PST_R2C, b.PST_FP32, B)
    plan.autotune("sg")
    import numpy as np
    u0 = np.stack([inputs.sg_gaussian(n, n, d, seed=s)[0] for s in range(B)])
    U0 = torch.from_numpy(u0).to("cuda", torch.float32)
    V0 = torch.zeros_like(U0)
    up, uc = torch.empty_like(U0), torch.empty_like(U0)
    plan.sg_start(U0, V0, up, uc, d, dt)
    h0 = plan.conserved_quantities("sg", up, uc, d=d, dt=dt)[:, 0]
    plan.sg_step(up, uc, d, dt, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.sg_step(up, uc, d, dt, steps - 11)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h1 = plan.conserved_quantities("sg", up, uc, d=d, dt=dt)[:, 0]
    plan.profile_enable(True)
    plan.sg_step(up, uc, d, dt, 20)
    r = plan.profile_read(b.PASS_SG_ROW)
    c = plan.profile_read(b.PASS_SG_COL)
    plan.profile_enable(False)
    rate = B * n * n * (steps - 11) / el
    return {"pt_steps_per_s": rate, "ms_per_step": el / (steps - 11) * 1e3,
            "alg_bytes_per_pt_step": 40, "pct_hbm_roofline": rate * 40 / (HBM_PEAK_GBS * 1e9),
            "row_us": r[0] / r[1] * 1e3, "col_us": c[0] / c[1] * 1e3,
            "max_rel_H_drift": float(np.max(np.abs(h1 / h0 - 1)))}


def bench_ns(b, inputs):
    """Navier-Stokes uneven batch: 4 x 1024^2 + 4 x 2048^2 FP32 random-phase
    vorticity, nu 1e-3, adaptive fixed point (tol 1e-10), through
    solve_batch.  dt 2.5e-4: at 1e-3 the scheme's fixed-point iteration
    diverges for these grids (it does in the FP64 oracle too), at 2.5e-4 it
    contracts in about 5 iterations per step.  The run is checked to stay
    finite and converged."""
    import torch
    steps, dt = 100, 2.5e-4
    fields = [torch.from_numpy(inputs.ns_random_phase(1024 if s < 4 else 2048, seed=s)).to("cuda", torch.float32)
              for s in range(8)]
    pr = b.make_params("ns", inputs.NS_DOMAIN, dt, nu=1e-3, tol=1e-10, max_iter=50)
    st = [torch.full((1,), -1, dtype=torch.int32, device="cuda") for _ in fields]
    reqs = [{"eq": "ns", "f0": f, "params": pr, "nsteps": 5, "dev_status": s} for f, s in zip(fields, st)]
    b.solve_batch(reqs)
    torch.cuda.synchronize()
    for r in reqs:
        r["nsteps"] = steps
    t0 = time.perf_counter()
    b.solve_batch(reqs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ok = all(int(s.item()) == b.PST_OK for s in st) and all(bool(torch.isfinite(f).all()) for f in fields)
    pts = 4 * (1024 ** 2 + 2048 ** 2) * steps
    return {"pt_steps_per_s": pts / el, "steps": steps, "dt": dt, "ms_per_step": el / steps * 1e3,
            "all_converged_and_finite": ok}


def time_nls(b, inputs, n, prec, batch, steps, dt=1e-3, variant=None, plans=1):
    """grid-pt-steps/s of NLS split steps: `plans` separate one-field plans
    stepped one after another (plain path) when plans > 1, else one plan of
    `batch` fields."""
    import torch
    d = inputs.PAPER_DOMAIN
    cdt = torch.complex64 if prec == b.PST_FP32 else torch.complex128
    psi0 = torch.from_numpy(inputs.nls_gaussian(n, n, d, seed=0)).to("cuda", cdt)
    if plans > 1:
        ps = [b.Plan(n, n, b.PST_C2C, prec, 1) for _ in range(plans)]
        fs = [psi0.reshape(1, n, n).clone() for _ in range(plans)]
        for p in ps:
            p.autotune("nls")
        run = lambda k: [p.nls_step(f, d, dt, 1.0, k) for p, f in zip(ps, fs)]
        pts = plans * n * n
    else:
        p = b.Plan(n, n, b.PST_C2C, prec, batch)
        if variant is None:
            p.autotune("nls")
        else:
            p.set_column_variant(variant)
        f = psi0.reshape(1, n, n).repeat(batch, 1, 1).contiguous()
        run = lambda k: p.nls_step(f, d, dt, 1.0, k)
        pts = batch * n * n
    run(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    return pts * steps / (time.perf_counter() - t0)


def bench_nls_cases(b, inputs):
    """Cases beside the headline: FP64 4096^2 and a batch of 4 x 4096^2
    FP32 (fields that cannot stay in the 256 MB last-level cache), batched vs
    plain stepping of 4 x 1024^2, and the headline with each column variant
    (the autotuner's candidates)."""
    out = {
        "nls_4096_fp64": time_nls(b, inputs, 4096, b.PST_FP64, 1, 100),
        "nls_4096x4_fp32": time_nls(b, inputs, 4096, b.PST_FP32, 4, 100),
        "nls_1024x4_fp32_batched": time_nls(b, inputs, 1024, b.PST_FP32, 4, 400),
        "nls_1024x4_fp32_plain": time_nls(b, inputs, 1024, b.PST_FP32, 1, 400, plans=4),
    }
    nv = len(b.column_variants(b.PST_FP32, 4096, True))
    out["nls_4096_fp32_by_column_variant"] = [time_nls(b, inputs, 4096, b.PST_FP32, 1, 200, variant=v)
                                              for v in range(nv)]
    out["unit"] = "grid-pt-steps/s"
    return out


def bench_sweep(b, inputs):
    """The paper's grid sweeps (its Tables 2-4 workloads), FP64 as in the
    paper and FP32: NLS 20 steps of 1e-5 on [-5pi,5pi)^2 (64^2-8192^2),
    sine-Gordon 500 steps of 1e-3 (64^2-4096^2), Navier-Stokes Taylor-Green
    20 steps of 1.25e-3 on [0,1)^2, nu 0.1, tol 1e-10 (64^2-4096^2).  Seconds
    for the paper's step count, loop only, one field, default tiles after
    autotuning."""
    import numpy as np
    import torch
    d = inputs.PAPER_DOMAIN
    res = {"nls": {}, "sg": {}, "ns": {}}
    for prec, name in ((b.PST_FP64, "fp64"), (b.PST_FP32, "fp32")):
        cdt = torch.complex128 if prec == b.PST_FP64 else torch.complex64
        rdt = torch.float64 if prec == b.PST_FP64 else torch.float32
        for e in range(6, 14):
            n = 1 << e
            p = b.Plan(n, n, b.PST_C2C, prec, 1)
            p.autotune("nls")
            f = torch.from_numpy(inputs.nls_gaussian(n, n, d, seed=0)).to("cuda", cdt).reshape(1, n, n)
            p.nls_step(f, d, 1e-5, 1.0, 20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.nls_step(f, d, 1e-5, 1.0, 20)
            torch.cuda.synchronize()
            res["nls"][f"{name}_{n}"] = time.perf_counter() - t0
            del p, f
        for e in range(6, 13):
            n = 1 << e
            p = b.Plan(n, n, b.PST_R2C, prec, 1)
            p.autotune("sg")
            u0 = torch.from_numpy(inputs.sg_gaussian(n, n, d, seed=0)[0]).to("cuda", rdt).reshape(1, n, n)
            up, uc = torch.empty_like(u0), torch.empty_like(u0)
            p.sg_start(u0, torch.zeros_like(u0), up, uc, d, 1e-3)
            p.sg_step(up, uc, d, 1e-3, 5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.sg_step(up, uc, d, 1e-3, 500)
            torch.cuda.synchronize()
            res["sg"][f"{name}_{n}"] = time.perf_counter() - t0
            del p, u0, up, uc
            p = b.Plan(n, n, b.PST_R2C, prec, 1)
            p.autotune("ns")
            w0 = torch.from_numpy(inputs.taylor_green(n, 0.0, 0.1)).to("cuda", rdt).reshape(1, n, n)
            w = w0.clone()
            p.ns_step(w, inputs.NS_DOMAIN, 1.25e-3, 0.1, 2, tol=1e-10)
            w.copy_(w0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.ns_step(w, inputs.NS_DOMAIN, 1.25e-3, 0.1, 20, tol=1e-10)
            torch.cuda.synchronize()
            res["ns"][f"{name}_{n}"] = time.perf_counter() - t0
            exact = inputs.taylor_green(n, 20 * 1.25e-3, 0.1)
            res["ns"][f"{name}_{n}_max_err"] = float(np.max(np.abs(w[0].double().cpu().numpy() - exact)))
            del p, w, w0
        torch.cuda.empty_cache()
    res["unit"] = "s for the paper's step count"
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=512, help="requests in the serving mix (0 = skip)")
    ap.add_argument("--extra", nargs="?", const="sg,ns,nls", default="",
                    help="also time sine-Gordon (sg) and Navier-Stokes (ns) batches and more NLS cases (nls); "
                         "a comma-separated subset, all three when given alone")
    ap.add_argument("--sweep", action="store_true", help="also run the paper's grid sweeps (Tables 2-4)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    extra = {x for x in args.extra.split(",") if x}
    if extra - {"sg", "ns", "nls"}:
        print(f"unknown --extra sections: {sorted(extra - {'sg', 'ns', 'nls'})}", file=sys.stderr)
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
    col_variant = plan.autotune("nls")
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
    progress(f"headline: {value:.4g} grid-pt-steps/s")

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
    traffic = traffic_from_profile(kname, col_variant) if (n, prec) == (4096, b.PST_FP32) else None

    # device-to-device copy bandwidth, for context (1 GiB each way: far larger
    # than the caches, also the calibration kernel for the HBM byte counters)
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 5 / (time.perf_counter() - t1) / 1e9
    del src, dst

    out = {
        "metric": "grid-pt-steps/s & %HBM roofline, 2D NLS 4096\u00b2; p50/p99 mixed-solve latency",
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
        "column_variant": col_variant,
        "copy_GBps": copy_gbs,
        "mass_rel_drift": float(q1[0, 0] / q0[0, 0] - 1),
        "energy_rel_drift": float(q1[0, 1] / q0[0, 1] - 1),
    }
    if "sg" in extra:
        out["sine_gordon_2048x16"] = bench_sg(b, inputs)
        progress("sine-Gordon section done")
    if "ns" in extra:
        out["navier_stokes_uneven"] = bench_ns(b, inputs)
        progress("Navier-Stokes section done")
    if "nls" in extra:
        out["nls_cases"] = bench_nls_cases(b, inputs)
        progress("NLS cases done")
    if args.sweep:
        out["paper_sweep"] = bench_sweep(b, inputs)
        progress("paper sweep done")
    if args.serve > 0:
        out["serving"] = bench_serve(args.serve)
        progress("serving done")
    if not args.no_cpu_baseline:
        cb, ref, ref_steps = cpu_baseline(n, dt)
        # the same steps on the device from the same initial field: max |gpu - oracle| / max |oracle|
        g0 = torch.from_numpy(inputs.nls_gaussian(n, n, d, seed=0)).to("cuda", plan.complex_dtype)
        g0 = g0.reshape(1, n, n).contiguous()
        plan.nls_step(g0, d, dt, g, ref_steps)
        got = g0[0].cpu().numpy()
        cb["gpu_vs_oracle"] = {"steps": ref_steps,
                               "max_rel_err": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))}
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
