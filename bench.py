"""Benchmark: 2D NLS split-step at 4096^2 on one MI355X, in the paper's double
precision, with the other workloads beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp64|fp32] [--n N]
                    [--no-cpu-baseline] [--serve COUNT] [--skip fp32,sg,ns,sweep,ablation]
                    [--sweep] [--extra [nls]]

Headline workload: a 4096^2 periodic grid on [-5pi,5pi)^2, psi0 = 0.5 exp(-r^2)
(1 + 0.01 xi) with seeded noise xi, dt = 1e-3, g = +1, complex128 fields (the
paper's Tables 2-4 are double precision; --prec fp32 makes complex64 the
headline).  A step is one Strang step: one row pass and one column pass over
the field.  K steps run in one nls_step call between two device
synchronisations; the field is resident in HBM before the timed region.

One JSON line on stdout carries:
  value / roofline      headline throughput (grid-point-steps/s) and the
                        dominant kernel's algorithmic bytes per launch over its
                        average launch duration (HIP events on the plan's
                        stream, in a second run of the same K steps);
  nls_4096_<other>      the same measurement in the other precision;
  sine_gordon_2048x16   16 seeds of 2048^2 FP32 in one plan, 500 steps;
  navier_stokes_uneven  4 x 1024^2 + 4 x 2048^2 FP32 through solve_batch;
  paper_sweep           the paper's Tables 2-4 workloads: the 4096^2 rows
                        and sine-Gordon 8192^2 (every grid with --sweep);
  autotune_ablation     default against autotuned tiles, every equation,
                        256^2-4096^2, FP64 and FP32;
  serving               the 512-request mix: p50/p99 latency, throughput,
                        against the plain one-request-at-a-time path;
  cpu_baseline          the FP64 oracle timed on the host's cores on a
                        bounded sample of the headline workload, with the
                        device field's deviation from it after the same steps.
Progress lines for finished sections go to stderr.  Every section's fraction
of the HBM roofline uses the algorithmic bytes per point of the method
(NLS 16 B per pass in FP32, 32 in FP64; sine-Gordon 20 + 12 per step; Navier-
Stokes 32 + 20 per fixed-point iteration) and the 8 TB/s peak.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# algorithmic bytes per grid point (FP32; FP64 doubles them)
NLS_PASS_BYTES = 16            # read + write of one complex value
SG_ROW_BYTES, SG_COL_BYTES = 20, 12   # the method's bytes (level form); the increment form moves 28 in the row pass
NS_COL_BYTES, NS_ROW_BYTES = 32, 20   # per fixed-point iteration; the increment form reads 4 more
SECTIONS = ("fp32", "sg", "ns", "sweep", "ablation")


def kernel_source_hash(files=("fft_line.hpp", "kernels.hpp", "k_nls.hip", "pst_common.hpp")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1206_3215_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


SG_SOURCES = ("fft_line.hpp", "kernels.hpp", "k_sg.hip", "pst_common.hpp")
NS_SOURCES = ("fft_line.hpp", "kernels.hpp", "k_ns.hip", "pst_common.hpp")


def traffic_from_profile(kernel: str, variant: int, name: str, sources=None):
    """HBM bytes per launch of one tile variant of a kernel, from a committed
    counter summary, if it was taken on the current kernel sources; None
    otherwise (or when that variant was not counted)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != (kernel_source_hash(sources) if sources else kernel_source_hash()):
        return None
    k = rec.get("kernels", {}).get(kernel, {}).get("variants", {}).get(str(variant))
    return None if k is None else k.get("bytes_per_launch")


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


def measure_nls(b, inputs, n, prec, K, W, traffic_file=None):
    """Throughput of K NLS steps in one call on an autotuned plan, then the
    per-pass average launch durations over a second run of K steps."""
    import torch
    d = inputs.PAPER_DOMAIN
    dt, g = 1e-3, 1.0
    plan = b.Plan(n, n, b.PST_C2C, prec, 1)
    plan.autotune("nls")
    row_variant, col_variant = plan.variants()
    psi = torch.from_numpy(inputs.nls_gaussian(n, n, d, seed=0)).to("cuda", plan.complex_dtype)
    psi = psi.reshape(1, n, n).contiguous()
    q0 = plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g)
    if W > 0:
        plan.nls_step(psi, d, dt, g, W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.nls_step(psi, d, dt, g, K)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    q1 = plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g)
    value = n * n * K / el
    plan.profile_enable(True)
    plan.nls_step(psi, d, dt, g, K)
    torch.cuda.synchronize()
    passes = {"nls_row": plan.profile_read(b.PASS_NLS_ROW), "nls_col": plan.profile_read(b.PASS_NLS_COL)}
    plan.profile_enable(False)
    assert plan.sync_status() == b.PST_OK, "NLS headline field is not finite"
    dom = max(passes, key=lambda k: passes[k][0])
    avg_s = passes[dom][0] / passes[dom][1] / 1e3
    esz = 1 if prec == b.PST_FP32 else 2
    alg_bytes = NLS_PASS_BYTES * esz * n * n
    achieved = alg_bytes / avg_s / 1e9
    kname = {"nls_row": "k_nls_row", "nls_col": "k_nls_col"}[dom]
    traffic = traffic_from_profile(kname, {"nls_row": row_variant, "nls_col": col_variant}[dom],
                                   traffic_file) if traffic_file else None
    out = {
        "value": value, "ms_per_step": el / K * 1e3,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
                     "avg_launch_us": avg_s * 1e6, "bytes_per_launch_alg": alg_bytes},
        "pct_hbm_roofline_step": value * 2 * NLS_PASS_BYTES * esz / (HBM_PEAK_GBS * 1e9),
        "passes_avg_us": {k: (v[0] / max(v[1], 1)) * 1e3 for k, v in passes.items()},
        "column_variant": col_variant, "row_variant": row_variant,
        "mass_rel_drift": float(q1[0, 0] / q0[0, 0] - 1),
        "energy_rel_drift": float(q1[0, 1] / q0[0, 1] - 1),
    }
    return out, plan


def bench_sg(b, inputs):
    """Sine-Gordon 2048^2 FP32, 16 seeds in one plan: start-up plus 499 steps
    of dt 0.01 (10 of them untimed warm-up)."""
    import numpy as np
    import torch
    n, B, dt, steps = 2048, 16, 0.01, 500
    d = inputs.PAPER_DOMAIN
    plan = b.Plan(n, n, b.PST_R2C, b.PST_FP32, B)
    variant = plan.autotune("sg")
    u0 = np.stack([inputs.sg_gaussian(n, n, d, seed=s)[0] for s in range(B)])
    U0 = torch.from_numpy(u0).to("cuda", torch.float32)
    V0 = torch.zeros_like(U0)
    up, uc = torch.empty_like(U0), torch.empty_like(U0)
    plan.sg_start(U0, V0, up, uc, d, dt)
    del U0, V0
    h0 = plan.conserved_quantities("sg", up, uc, d=d, dt=dt)[:, 0]
    plan.sg_step(up, uc, d, dt, 10)
    torch.cuda.synchronize()
    timed = steps - 11
    t0 = time.perf_counter()
    plan.sg_step(up, uc, d, dt, timed)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h1 = plan.conserved_quantities("sg", up, uc, d=d, dt=dt)[:, 0]
    plan.profile_enable(True)
    plan.sg_step(up, uc, d, dt, 50)
    r = plan.profile_read(b.PASS_SG_ROW)
    c = plan.profile_read(b.PASS_SG_COL)
    plan.profile_enable(False)
    assert plan.sync_status() == b.PST_OK
    pts = B * n * n
    rate = pts * timed / el
    row_s, col_s = r[0] / r[1] / 1e3, c[0] / c[1] / 1e3
    row_alg, col_alg = SG_ROW_BYTES * pts, SG_COL_BYTES * pts
    rt = traffic_from_profile("k_sg_row", 0, "sg_2048x16_fp32_traffic.json", SG_SOURCES)
    ct = traffic_from_profile("k_sg_col", variant, "sg_2048x16_fp32_traffic.json", SG_SOURCES)
    return {"pt_steps_per_s": rate, "ms_per_step": el / timed * 1e3, "steps_timed": timed,
            "alg_bytes_per_pt_step": SG_ROW_BYTES + SG_COL_BYTES,
            "pct_hbm_roofline_step": rate * (SG_ROW_BYTES + SG_COL_BYTES) / (HBM_PEAK_GBS * 1e9),
            "row": {"avg_launch_us": row_s * 1e6, "bytes_per_launch_alg": row_alg,
                    "frac": row_alg / row_s / 1e9 / HBM_PEAK_GBS, "traffic": rt},
            "col": {"avg_launch_us": col_s * 1e6, "bytes_per_launch_alg": col_alg,
                    "frac": col_alg / col_s / 1e9 / HBM_PEAK_GBS, "traffic": ct},
            "column_variant": variant,
            "max_rel_H_drift": float(np.max(np.abs(h1 / h0 - 1)))}


def bench_ns(b, inputs):
    """Navier-Stokes uneven batch: 4 x 1024^2 + 4 x 2048^2 FP32 random-phase
    vorticity, nu 1e-3, adaptive fixed point (tol 1e-10), through
    solve_batch.  dt 2.5e-4: at 1e-3 the scheme's fixed-point iteration
    diverges for these grids (it does in the FP64 oracle too), at 2.5e-4 it
    contracts in a few iterations per step.  The iterations per step come
    from the same fields stepped on single-size plans (untimed)."""
    import torch
    steps, dt = 100, 2.5e-4
    sizes = [1024] * 4 + [2048] * 4
    host = [inputs.ns_random_phase(n, seed=s) for s, n in enumerate(sizes)]
    fields = [torch.from_numpy(w).to("cuda", torch.float32) for w in host]
    pr = b.make_params("ns", inputs.NS_DOMAIN, dt, nu=1e-3, tol=1e-10, max_iter=50)
    st = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in fields]
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
    # iterations per step of the same trajectories (fields after the 5 warm-up steps)
    iters = []
    for n in (1024, 2048):
        sel = [i for i, m in enumerate(sizes) if m == n]
        plan = b.Plan(n, n, b.PST_R2C, b.PST_FP32, len(sel))
        w = torch.stack([torch.from_numpy(host[i]).to("cuda", torch.float32) for i in sel])
        its = torch.zeros((5 + steps) * len(sel), dtype=torch.int32, device="cuda")
        plan.ns_step(w, inputs.NS_DOMAIN, dt, 1e-3, 5 + steps, tol=1e-10, max_iter=50, dev_iters=its)
        iters.append(float(its.view(-1, len(sel))[5:].float().mean().item()))
        del plan, w
    pts_1k, pts_2k = 4 * 1024 ** 2, 4 * 2048 ** 2
    pt_iters = (pts_1k * iters[0] + pts_2k * iters[1]) * steps
    return {"pt_steps_per_s": (pts_1k + pts_2k) * steps / el, "pt_iters_per_s": pt_iters / el, "steps": steps,
            "dt": dt, "ms_per_step": el / steps * 1e3, "iters_per_step": {"1024": iters[0], "2048": iters[1]},
            "alg_bytes_per_pt_iter": NS_COL_BYTES + NS_ROW_BYTES,
            "pct_hbm_roofline": pt_iters / el * (NS_COL_BYTES + NS_ROW_BYTES) / (HBM_PEAK_GBS * 1e9),
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
    """Cases beside the headline: a batch of 4 x 4096^2 FP32 (fields that
    cannot stay in the 256 MB last-level cache), batched vs plain stepping of
    4 x 1024^2, and 4096^2 FP32 and FP64 with each column variant."""
    out = {
        "nls_4096x4_fp32": time_nls(b, inputs, 4096, b.PST_FP32, 4, 100),
        "nls_1024x4_fp32_batched": time_nls(b, inputs, 1024, b.PST_FP32, 4, 400),
        "nls_1024x4_fp32_plain": time_nls(b, inputs, 1024, b.PST_FP32, 1, 400, plans=4),
    }
    for prec, name in ((b.PST_FP32, "fp32"), (b.PST_FP64, "fp64")):
        nv = len(b.column_variants(prec, 4096, True))
        out[f"nls_4096_{name}_by_column_variant"] = [time_nls(b, inputs, 4096, prec, 1, 200, variant=v)
                                                     for v in range(nv)]
    out["unit"] = "grid-pt-steps/s"
    return out


def bench_sweep(b, inputs, full: bool):
    """The paper's grid sweeps (its Tables 2-4 workloads), FP64 as in the
    paper and FP32: NLS 20 steps of 1e-5 on [-5pi,5pi)^2, sine-Gordon 500
    steps of 1e-3, Navier-Stokes Taylor-Green 20 steps of 1.25e-3 on [0,1)^2,
    nu 0.1, tol 1e-10, with the max error against the exact vortex (Table 4
    prints 1.65e-5 for every grid).  Seconds for the paper's step count, loop
    only, one field, autotuned tiles.  Grids: every size of the tables with
    full, else the 4096^2 row of each table and sine-Gordon 8192^2."""
    import numpy as np
    import torch
    d = inputs.PAPER_DOMAIN
    nls_sizes = [1 << e for e in range(6, 14)] if full else [4096]
    sg_sizes = [1 << e for e in range(6, 14)] if full else [4096, 8192]
    ns_sizes = [1 << e for e in range(6, 13)] if full else [4096]
    res = {"nls": {}, "sg": {}, "ns": {}}
    for prec, name in ((b.PST_FP64, "fp64"), (b.PST_FP32, "fp32")):
        cdt = torch.complex128 if prec == b.PST_FP64 else torch.complex64
        rdt = torch.float64 if prec == b.PST_FP64 else torch.float32
        for n in nls_sizes:
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
        for n in sg_sizes:
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
        for n in ns_sizes:
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
    res["paper_best_gpu_s_4096"] = {"nls": 1.49, "sg": 16.53, "ns": 5.814,
                                    "hardware": "Tesla M2070, FP64 (Tables 2-4)"}
    return res


def bench_ablation(b, inputs, sizes=(256, 512, 1024, 2048, 4096)):
    """Autotuner ablation: grid-pt-steps/s of one field with the default
    tiles (row and column variant 0) against the autotuned ones, for each
    equation, size and precision.  NLS 40 steps of dt 1e-3; sine-Gordon 40
    steps of dt 1e-3; Navier-Stokes (Taylor-Green, nu 0.1, dt 1.25e-3) 8
    steps of exactly 3 fixed-point iterations, so both sides do the same
    work."""
    import torch
    d = inputs.PAPER_DOMAIN
    out = {}
    for prec, pname in ((b.PST_FP64, "fp64"), (b.PST_FP32, "fp32")):
        cdt = torch.complex128 if prec == b.PST_FP64 else torch.complex64
        rdt = torch.float64 if prec == b.PST_FP64 else torch.float32
        for eq in ("nls", "sg", "ns"):
            for n in sizes:
                rates = {}
                for mode in ("default", "autotuned"):
                    p = b.Plan(n, n, b.PST_C2C if eq == "nls" else b.PST_R2C, prec, 1)
                    if mode == "autotuned":
                        p.autotune(eq)
                    if eq == "nls":
                        f = torch.from_numpy(inputs.nls_gaussian(n, n, d, seed=0)).to("cuda", cdt).reshape(1, n, n)
                        run = lambda k, p=p, f=f: p.nls_step(f, d, 1e-3, 1.0, k)
                        k = 40
                    elif eq == "sg":
                        u = torch.from_numpy(inputs.sg_gaussian(n, n, d, seed=0)[0]).to("cuda", rdt).reshape(1, n, n)
                        v = u.clone()
                        run = lambda k, p=p, u=u, v=v: p.sg_step(u, v, d, 1e-3, k)
                        k = 40
                    else:
                        w = torch.from_numpy(inputs.taylor_green(n, 0.0, 0.1)).to("cuda", rdt).reshape(1, n, n)
                        run = lambda k, p=p, w=w: p.ns_step(w, inputs.NS_DOMAIN, 1.25e-3, 0.1, k, fixed_iters=3)
                        k = 8
                    run(2)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    run(k)
                    torch.cuda.synchronize()
                    rates[mode] = n * n * k / (time.perf_counter() - t0)
                    if mode == "autotuned":
                        rates["variants"] = list(p.variants())
                    del p
                rates["speedup"] = rates["autotuned"] / rates["default"]
                out[f"{eq}_{n}_{pname}"] = rates
    out["unit"] = "grid-pt-steps/s (NS: steps of 3 fixed-point iterations)"
    return out


def bench_serve(count: int):
    """Serving mix: Poisson arrivals, equation uniform over {NLS, SG, NS},
    n = 2^e with e uniform on 7..11, steps uniform on 100..2000, FP32.
    The arrival rate is set to 0.8x the batched capacity measured on the same
    mix served all at once; p50/p99 latency and throughput are then measured
    with real-time arrivals (requests advance by 64 steps per round, one
    more such chunk per 0.25 s waited), and the plain one-at-a-time path is timed on the
    same requests: its p50/p99 are those of a first-in-first-out queue with
    the same arrival times and each request's measured solve time."""
    import numpy as np
    import torch

    from paper_1206_3215_amd import inputs
    from paper_1206_3215_amd.serve import GpuExecutor, Server, fifo_baseline, fifo_latencies
    budget = 16 << 30
    mix0 = inputs.serving_mix(count, rate_hz=1.0)
    work = sum(r.n * r.n * r.steps for r in mix0)
    ex = GpuExecutor()
    cap_rep = Server(ex, budget, chunk=64).run(mix0, realtime=False)
    cap = cap_rep.summary()
    rate = 0.8 * cap["pt_steps_per_s"] / (work / count)
    mix = inputs.serving_mix(count, rate_hz=rate)
    server = Server(ex, budget, chunk=64, age_s=0.25, max_boost=64)
    # a real-time warm-up on the first quarter of the mix: the first real-time
    # pass meets allocations and chunk schedules the capacity run did not
    server.run(mix[: max(1, count // 4)], realtime=True)
    rep = server.run(mix, realtime=True)
    summ = rep.summary()
    fifo_wall, fifo_rate, _, service = fifo_baseline(mix)
    torch.cuda.synchronize()
    # the plain path's latencies under the same arrivals: one request at a
    # time in arrival order, each taking its measured solve time
    fifo_lat = list(fifo_latencies(mix, service).values())
    return {"requests": count, "hbm_budget_GiB": budget / 2 ** 30, "arrival_rate_hz": rate,
            "batched_capacity_pt_steps_per_s": cap["pt_steps_per_s"],
            "pt_steps_per_s": summ["pt_steps_per_s"], "p50_latency_s": summ["p50_latency_s"],
            "p99_latency_s": summ["p99_latency_s"], "wall_s": summ["wall_s"],
            "statuses_ok": all(j.status == 0 for j in rep.jobs),
            "fifo_pt_steps_per_s": fifo_rate, "fifo_wall_s": fifo_wall,
            "fifo_p50_latency_s": float(np.percentile(fifo_lat, 50)),
            "fifo_p99_latency_s": float(np.percentile(fifo_lat, 99)),
            "batched_over_fifo": cap["pt_steps_per_s"] / fifo_rate}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=512, help="requests in the serving mix (0 = skip)")
    ap.add_argument("--skip", default="", help=f"comma-separated sections to leave out: {','.join(SECTIONS)}")
    ap.add_argument("--sweep", action="store_true", help="run the paper's sweeps over every grid (Tables 2-4)")
    ap.add_argument("--extra", nargs="?", const="nls", default="",
                    help="also time more NLS cases (nls): 4 x 4096^2, batched vs plain, column variants")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    skip = {x for x in args.skip.split(",") if x}
    extra = {x for x in args.extra.split(",") if x}
    if skip - set(SECTIONS) or extra - {"nls"}:
        print(f"unknown sections: {sorted((skip - set(SECTIONS)) | (extra - {'nls'}))}", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1206_3215_amd import binding as b
    from paper_1206_3215_amd import inputs

    torch.cuda.set_device(0)
    n, K, W = args.n, args.steps, args.warmup
    prec = b.PST_FP64 if args.prec == "fp64" else b.PST_FP32
    other, oname = (b.PST_FP32, "fp32") if prec == b.PST_FP64 else (b.PST_FP64, "fp64")
    sub = {}
    if "fp32" not in skip:
        sub[f"nls_{n}_{oname}"], p = measure_nls(b, inputs, n, other, K, W, f"nls_{n}_{oname}_traffic.json")
        del p
        progress(f"NLS {oname}: {sub[f'nls_{n}_{oname}']['value']:.4g} grid-pt-steps/s")
    head, plan = measure_nls(b, inputs, n, prec, K, W, f"nls_{n}_{args.prec}_traffic.json")
    progress(f"headline NLS {args.prec}: {head['value']:.4g} grid-pt-steps/s")

    # device-to-device copy bandwidth, for context (1 GiB each way: far larger
    # than the caches)
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
        "metric": "grid-pt-steps/s & %HBM roofline, 2D NLS 4096²; p50/p99 mixed-solve latency",
        "value": head["value"],
        "unit": "grid-pt-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == b.PST_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"nls_split_step_{n}x{n}_{args.prec}", "grid": [n, n],
                   "domain": "[-5pi,5pi)^2", "dt": 1e-3, "g": 1.0, "ic": "0.5exp(-r^2)(1+0.01xi), seed 0"},
        "roofline": head["roofline"],
        "pct_hbm_roofline_step": head["pct_hbm_roofline_step"],
        "passes_avg_us": head["passes_avg_us"],
        "column_variant": head["column_variant"],
        "row_variant": head["row_variant"],
        "copy_GBps": copy_gbs,
        "mass_rel_drift": head["mass_rel_drift"],
        "energy_rel_drift": head["energy_rel_drift"],
    }
    out.update(sub)
    if "sg" not in skip:
        out["sine_gordon_2048x16_fp32"] = bench_sg(b, inputs)
        progress("sine-Gordon section done")
    if "ns" not in skip:
        out["navier_stokes_uneven_fp32"] = bench_ns(b, inputs)
        progress("Navier-Stokes section done")
    if "nls" in extra:
        out["nls_cases"] = bench_nls_cases(b, inputs)
        progress("NLS cases done")
    if "sweep" not in skip or args.sweep:
        out["paper_sweep"] = bench_sweep(b, inputs, full=args.sweep)
        progress("paper sweep done")
    if "ablation" not in skip:
        out["autotune_ablation"] = bench_ablation(b, inputs)
        progress("autotuner ablation done")
    if args.serve > 0:
        out["serving"] = bench_serve(args.serve)
        progress("serving done")
    if not args.no_cpu_baseline:
        cb, ref, ref_steps = cpu_baseline(n, 1e-3)
        # the same steps on the device from the same initial field: max |gpu - oracle| / max |oracle|
        g0 = torch.from_numpy(inputs.nls_gaussian(n, n, inputs.PAPER_DOMAIN, seed=0)).to("cuda", plan.complex_dtype)
        g0 = g0.reshape(1, n, n).contiguous()
        plan.nls_step(g0, inputs.PAPER_DOMAIN, 1e-3, 1.0, ref_steps)
        got = g0[0].cpu().numpy()
        cb["gpu_vs_oracle"] = {"steps": ref_steps, "precision": args.prec,
                               "max_rel_err": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))}
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
