"""Reference samples of the full-length workloads, computed by the FP64 oracle.

    python tests/golden/gen_refs.py [nls] [sg] [ns] [twin]

Each section runs the oracle (``oracle/``) on the seeded inputs of
``paper_1206_3215_amd/inputs.py`` and writes a compressed ``.npz`` of
samples beside this script; the GPU parity tests read the index sets stored
in the file, take the same points from the device result and compare them
element by element.  Nothing here runs or reads the HIP path.

Sampling of an n-by-n field (every sample index is stored in the file):
  * full rows and full columns at 0, 1, n/2 - 1, n/2, n - 1;
  * a 128 x 128 lattice with stride n/128 (offsets 3 in y, 5 in x);
  * a dense central window (the workloads' pulses sit at the centre).

Sections:
  nls   NLS 4096^2 on [-5pi,5pi)^2, psi0 = 0.5 exp(-r^2)(1 + 0.01 xi), seed 0,
        dt 1e-3, g = +1, 1000 Strang steps (the headline workload); mass and
        energy every 100 steps.  About 15 minutes on 8 cores.
  sg    sine-Gordon 2048^2 on [-5pi,5pi)^2, u0 = 0.5 exp(-r^2) + 1e-3 xi,
        v0 = 0, dt 0.01: start-up plus 499 steps (u^499, u^500) for seeds 0
        and 11 of the 16-seed batch; Hamiltonian H^{1/2} and H^{499+1/2}.
  twin  Navier-Stokes predictability horizon: the oracle against itself
        started from a perturbed field (relative 1e-14 and 1e-7 of
        max |omega|), 1024^2 random-phase seed 0, nu 1e-3, dt 2.5e-4,
        tol 1e-10, relative difference per step (JSON).
  ns    Navier-Stokes uneven batch: seeds 0-3 at 1024^2 and 4-7 at 2048^2,
        same parameters, samples at the steps named in NS_STEPS (inside the
        horizon measured by `twin`), with energy, enstrophy and iteration
        counts per step.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import nls as onls  # noqa: E402
from oracle import ns as ons  # noqa: E402
from oracle import sg as osg  # noqa: E402
from paper_1206_3215_amd import inputs  # noqa: E402

NLS_N, NLS_DT, NLS_STEPS = 4096, 1e-3, 1000
SG_N, SG_DT, SG_STEPS, SG_SEEDS = 2048, 0.01, 499, (0, 11)
NS_DT, NS_NU, NS_TOL, NS_MAXIT = 2.5e-4, 1e-3, 1e-10, 50
NS_SIZES = {0: 1024, 1: 1024, 2: 1024, 3: 1024, 4: 2048, 5: 2048, 6: 2048, 7: 2048}
NS_STEPS = (40, 240)
TWIN_STEPS = 240


def sample_spec(n: int, window: int) -> dict:
    lines = np.array(sorted({0, 1, n // 2 - 1, n // 2, n - 1}), dtype=np.int64)
    s = max(1, n // 128)
    return {"lines": lines, "lat_y": np.arange(3, n, s)[:128], "lat_x": np.arange(5, n, s)[:128],
            "win0": np.int64(n // 2 - window // 2), "win": np.int64(window)}


def take(f: np.ndarray, spec: dict, prefix: str) -> dict:
    w0, w = int(spec["win0"]), int(spec["win"])
    return {f"{prefix}rows": f[spec["lines"], :], f"{prefix}cols": f[:, spec["lines"]],
            f"{prefix}lat": f[np.ix_(spec["lat_y"], spec["lat_x"])],
            f"{prefix}win": f[w0:w0 + w, w0:w0 + w], f"{prefix}maxabs": np.max(np.abs(f))}


def log(msg: str) -> None:
    print(f"[gen_refs] {msg}", flush=True)


def gen_nls() -> None:
    d = inputs.PAPER_DOMAIN
    psi = inputs.nls_gaussian(NLS_N, NLS_N, d, seed=0)
    spec = sample_spec(NLS_N, 256)
    series = [(0, onls.mass(psi, d.lx, d.ly), onls.energy(psi, d.lx, d.ly, 1.0))]
    t0 = time.time()
    for k in range(1, NLS_STEPS + 1):
        psi = onls.step(psi, d.lx, d.ly, NLS_DT, 1.0)
        if k % 100 == 0:
            series.append((k, onls.mass(psi, d.lx, d.ly), onls.energy(psi, d.lx, d.ly, 1.0)))
            log(f"nls step {k} ({time.time() - t0:.0f} s)")
    out = dict(spec)
    out.update(take(psi, spec, "psi_"))
    out.update({"n": NLS_N, "dt": NLS_DT, "steps": NLS_STEPS, "g": 1.0, "seed": 0,
                "series": np.array(series, dtype=np.float64)})
    np.savez_compressed(os.path.join(HERE, "ref_nls_4096_1000.npz"), **out)


def gen_sg() -> None:
    d = inputs.PAPER_DOMAIN
    spec = sample_spec(SG_N, 128)
    out = dict(spec)
    out.update({"n": SG_N, "dt": SG_DT, "steps": SG_STEPS, "seeds": np.array(SG_SEEDS)})
    for s in SG_SEEDS:
        u0, v0 = inputs.sg_gaussian(SG_N, SG_N, d, seed=s)
        u1 = osg.start(u0, v0, d.lx, d.ly, SG_DT)
        h0 = osg.hamiltonian(u0, u1, d.lx, d.ly, SG_DT)
        t0 = time.time()
        a, b = osg.run(u0, u1, d.lx, d.ly, SG_DT, SG_STEPS)
        h1 = osg.hamiltonian(a, b, d.lx, d.ly, SG_DT)
        log(f"sg seed {s}: {time.time() - t0:.0f} s, H {h0[3]:.12g} -> {h1[3]:.12g}")
        out.update(take(a, spec, f"s{s}_prev_"))
        out.update(take(b, spec, f"s{s}_curr_"))
        out[f"s{s}_H0"] = np.array(h0)
        out[f"s{s}_H1"] = np.array(h1)
    np.savez_compressed(os.path.join(HERE, "ref_sg_2048_500.npz"), **out)


def rel_diff(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def gen_twin() -> None:
    n, seed = 1024, 0
    w0 = inputs.ns_random_phase(n, seed=seed)
    xi = inputs.noise(n, n, 1000 + seed)
    amp = np.max(np.abs(w0))
    runs = {"ref": w0.copy(), "p1e-14": w0 + 1e-14 * amp * xi, "p1e-7": w0 + 1e-7 * amp * xi}
    curves = {"p1e-14": [], "p1e-7": []}
    iters = []
    t0 = time.time()
    for k in range(1, TWIN_STEPS + 1):
        for key in runs:
            runs[key], it, ok = ons.step(runs[key], 1.0, 1.0, NS_DT, NS_NU, NS_TOL, NS_MAXIT)
            assert ok, (key, k)
            if key == "ref":
                iters.append(it)
        for key in curves:
            curves[key].append(rel_diff(runs[key], runs["ref"]))
        if k % 20 == 0:
            log(f"twin step {k} ({time.time() - t0:.0f} s): "
                + ", ".join(f"{key} {curves[key][-1]:.3e}" for key in curves))
    rec = {"workload": f"NS random-phase {n}^2 seed {seed}, nu {NS_NU}, dt {NS_DT}, tol {NS_TOL}, adaptive",
           "perturbation": "w0 + eps * max|w0| * xi, xi = inputs.noise(n, n, 1000 + seed)",
           "metric": "max|w_pert - w_ref| / max|w_ref| after each step",
           "steps": TWIN_STEPS, "iterations_ref": iters, "rel_diff": curves}
    with open(os.path.join(HERE, "ns_twin_1024.json"), "w") as fh:
        json.dump(rec, fh, indent=1)


def gen_ns() -> None:
    out = {"dt": NS_DT, "nu": NS_NU, "tol": NS_TOL, "max_iter": NS_MAXIT, "steps": np.array(NS_STEPS),
           "seeds": np.array(sorted(NS_SIZES))}
    for seed, n in NS_SIZES.items():
        w = inputs.ns_random_phase(n, seed=seed)
        spec = sample_spec(n, 64)
        out.update({f"s{seed}_{k}": v for k, v in spec.items()})
        out[f"s{seed}_n"] = n
        series, its = [(0, ons.energy(w, 1.0, 1.0), ons.enstrophy(w, 1.0, 1.0))], []
        t0 = time.time()
        for k in range(1, max(NS_STEPS) + 1):
            w, it, ok = ons.step(w, 1.0, 1.0, NS_DT, NS_NU, NS_TOL, NS_MAXIT)
            assert ok, (seed, k)
            its.append(it)
            series.append((k, ons.energy(w, 1.0, 1.0), ons.enstrophy(w, 1.0, 1.0)))
            if k in NS_STEPS:
                out.update(take(w, spec, f"s{seed}_t{k}_"))
        log(f"ns seed {seed} ({n}^2): {time.time() - t0:.0f} s, iterations {its[:8]}...")
        out[f"s{seed}_series"] = np.array(series)
        out[f"s{seed}_iters"] = np.array(its)
    np.savez_compressed(os.path.join(HERE, "ref_ns_uneven.npz"), **out)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["twin", "sg", "ns", "nls"]
    gens = {"nls": gen_nls, "sg": gen_sg, "ns": gen_ns, "twin": gen_twin}
    for name in todo:
        gens[name]()
        log(f"{name} done")
