"""Continuous-batching request loop for mixed pseudospectral solves.

Requests (equation, grid, steps, arrival time) arrive over time.  The server
keeps every admitted simulation's fields resident on the device and advances
all of them together, a chunk of at most `chunk` steps at a time, through
one `solve_batch` call per chunk (the library groups them by size class).
Between chunks it admits the requests that have arrived, as long as their
device footprint fits the memory budget, and retires the finished ones
(result copied to the host, latency stamped).  A GPU worker thread runs the
chunks while the main thread handles arrivals, so admission work (initial
conditions, host-to-device copies) overlaps with device work.

Executors implement the device side:
    footprint(req) -> bytes      (reserved while the request is admitted)
    admit(req) -> state          (allocate fields, write the initial condition)
    advance([(state, nsteps)])   (one batched call, returns when done; may
                                  return one status per work item)
    fetch(state) -> (np.ndarray, status)   (result on the host)
    release(state)
and optionally
    overhead_bytes() -> bytes    (device memory held beyond the admitted
                                  requests' reservations, read between chunks)
    trim()                       (give that memory back)
A request's status is the worst one reported for it over all its chunks
(NONFINITE outranks NOT_CONVERGED, which outranks OK).  `GpuExecutor` is the
MI355X one; tests drive the same loop with a CPU one.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np

from . import inputs

# Device bytes per grid point, FP32 (FP64 doubles them).  Fields of the
# request: NLS psi (8); sine-Gordon the two levels plus u0, v0 until the
# start-up step (16); Navier-Stokes omega (4).  Workspace each field takes in
# the library's cached plan of its size class (solve_batch): the C2C
# spectrum (8), or 4 half spectra and 4 derivative hybrids (32).
FIELD_BYTES_PER_POINT = {"nls": 8, "sg": 16, "ns": 4}
WORKSPACE_BYTES_PER_POINT = {"nls": 8, "sg": 32, "ns": 32}
# Admission reserves the fields and twice the workspace: a size class's
# cached plan has room for the next power of two of its group size, so the
# plans of the admitted requests' classes never exceed this reservation.
BYTES_PER_POINT = {eq: FIELD_BYTES_PER_POINT[eq] + 2 * WORKSPACE_BYTES_PER_POINT[eq]
                   for eq in FIELD_BYTES_PER_POINT}


def worst_status(a: int, b: int) -> int:
    """Latch: NONFINITE (6) outranks NOT_CONVERGED (5), which outranks OK."""
    return max(int(a), int(b))


@dataclasses.dataclass
class ServeParams:
    nls_dt: float = 1e-3
    sg_dt: float = 0.01
    # random-phase NS: at dt 1e-3 the scheme's fixed point diverges from 512^2 up;
    # at 2.5e-4 it contracts (about 5 iterations per step)
    ns_dt: float = 2.5e-4
    ns_nu: float = 1e-3
    ns_tol: float = 1e-10
    ns_max_iter: int = 30


@dataclasses.dataclass
class Job:
    req: inputs.Request
    state: object = None
    remaining: int = 0
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: np.ndarray | None = None
    status: int = 0


@dataclasses.dataclass
class Report:
    jobs: list
    wall_s: float
    pt_steps: float

    @property
    def latencies(self):
        return np.array([j.t_done - j.req.arrival_s for j in self.jobs])

    def summary(self) -> dict:
        lat = self.latencies
        return {"requests": len(self.jobs), "wall_s": self.wall_s,
                "pt_steps_per_s": self.pt_steps / self.wall_s if self.wall_s > 0 else 0.0,
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_latency_s": float(np.mean(lat))}


class Server:
    """Continuous batching: every admitted request advances by up to `chunk`
    steps per round, all of them in one executor call.  With age_s set, a
    request that has waited a seconds since its arrival advances by
    chunk * min(max_boost, 1 + a / age_s) steps instead, so the rounds drift
    from sharing the device equally (which stretches the largest requests)
    towards serving the oldest first."""

    def __init__(self, executor, budget_bytes: int, chunk: int = 50, age_s: float | None = None,
                 max_boost: int = 8):
        self.ex = executor
        self.budget = budget_bytes
        self.chunk = chunk
        self.age_s = age_s
        self.max_boost = max_boost

    def run(self, requests, realtime: bool = True) -> Report:
        """Serve `requests` (arrival_s relative to the start).  With
        realtime=False every request is treated as arrived at t = 0."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting: collections.deque = collections.deque()
        active: list[Job] = []
        done: list[Job] = []
        used = 0
        overhead = 0  # executor memory beyond the reservations, read between chunks
        lock = threading.Lock()
        t0 = time.perf_counter()
        now = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))

        for r in requests:
            if self.ex.footprint(r) > self.budget:
                raise ValueError(f"request {r.rid} needs more than the whole budget")

        def admit_ready():
            nonlocal used
            t = now()
            while pending and pending[0].arrival_s <= t:
                waiting.append(pending.popleft())
            while waiting and used + overhead + self.ex.footprint(waiting[0]) <= self.budget:
                r = waiting.popleft()
                job = Job(r, remaining=r.steps)
                job.state = self.ex.admit(r)
                job.t_admit = time.perf_counter() - t0
                used += self.ex.footprint(r)
                with lock:
                    active.append(job)

        def retire():
            nonlocal used
            with lock:
                finished = [j for j in active if j.remaining == 0]
            for j in finished:
                j.result, st = self.ex.fetch(j.state)
                j.status = worst_status(j.status, st)
                j.t_done = time.perf_counter() - t0
                self.ex.release(j.state)
                used -= self.ex.footprint(j.req)
                with lock:
                    active.remove(j)
                done.append(j)

        def refresh_overhead():
            # only between chunks: the executor may have to wait for the device
            nonlocal overhead
            if hasattr(self.ex, "overhead_bytes"):
                overhead = self.ex.overhead_bytes()
                if overhead and waiting and used + overhead + self.ex.footprint(waiting[0]) > self.budget \
                        and hasattr(self.ex, "trim"):
                    self.ex.trim()
                    overhead = self.ex.overhead_bytes()

        while pending or waiting or active:
            retire()
            refresh_overhead()
            admit_ready()
            with lock:
                batch = [j for j in active if j.remaining > 0]
            if not batch:
                if active:
                    continue  # zero-step jobs: retired at the top of the loop
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival_s - now())))
                continue
            if self.age_s:
                t = time.perf_counter() - t0
                boost = [min(self.max_boost, 1 + int(max(0.0, t - j.req.arrival_s) / self.age_s)) for j in batch]
            else:
                boost = [1] * len(batch)
            work = [(j.state, min(self.chunk * w, j.remaining)) for j, w in zip(batch, boost)]
            # the device advances this chunk while arrivals are admitted
            errors = []
            statuses = []

            def chunk():
                try:
                    statuses.append(self.ex.advance(work))
                except BaseException as e:  # re-raised on the main thread
                    errors.append(e)

            worker = threading.Thread(target=chunk)
            worker.start()
            while worker.is_alive():
                admit_ready()
                worker.join(timeout=0.002)
            if errors:
                raise errors[0]
            per_item = statuses[0] if statuses and statuses[0] is not None else [0] * len(batch)
            for j, (_, k), st in zip(batch, work, per_item):
                j.remaining -= k
                j.status = worst_status(j.status, st)
        wall = time.perf_counter() - t0
        pts = float(sum(j.req.n * j.req.n * j.req.steps for j in done))
        return Report(sorted(done, key=lambda j: j.req.rid), wall, pts)


# ----------------------------------------------------------------------------
# MI355X executor

def initial_condition(req: inputs.Request):
    """Seeded initial fields of a request (float64 / complex128, host)."""
    if req.eq == "nls":
        return (inputs.nls_gaussian(req.n, req.n, inputs.PAPER_DOMAIN, seed=req.rid),)
    if req.eq == "sg":
        u0, v0 = inputs.sg_gaussian(req.n, req.n, inputs.PAPER_DOMAIN, seed=req.rid)
        return u0, v0
    return (inputs.ns_random_phase(req.n, seed=req.rid),)


class GpuExecutor:
    """Fields live in torch tensors on cuda:0; every chunk is one solve_batch."""

    def __init__(self, params: ServeParams | None = None, fp64: bool = False):
        import torch

        from . import binding
        self.torch = torch
        self.b = binding
        self.p = params or ServeParams()
        self.rdt = torch.float64 if fp64 else torch.float32
        self.cdt = torch.complex128 if fp64 else torch.complex64
        self.stream = torch.cuda.Stream()          # default priority
        self.copy_stream = torch.cuda.Stream()
        self._sg_plans = {}
        self._classes = {}  # (eq, n) -> admitted requests of that size class
        p = self.p
        self.params = {
            "nls": binding.make_params("nls", inputs.PAPER_DOMAIN, p.nls_dt, g=1.0),
            "sg": binding.make_params("sg", inputs.PAPER_DOMAIN, p.sg_dt),
            "ns": binding.make_params("ns", inputs.NS_DOMAIN, p.ns_dt, nu=p.ns_nu, tol=p.ns_tol,
                                      max_iter=p.ns_max_iter),
        }

    def footprint(self, req) -> int:
        scale = 2 if self.rdt == self.torch.float64 else 1
        return BYTES_PER_POINT[req.eq] * req.n * req.n * scale

    def overhead_bytes(self) -> int:
        """Device memory beyond the admitted requests' reservations: cached
        batch plans of size classes without admitted requests (the others
        are covered by the reservations) and the sine-Gordon start-up plans'
        workspaces."""
        cache = self.b.batch_cache_bytes()
        reserved = sum(2 * WORKSPACE_BYTES_PER_POINT[eq] * n * n * (2 if self.rdt == self.torch.float64 else 1)
                       for eq, n in self._active_classes)
        start = sum(int(p.workspace.numel()) for p in self._sg_plans.values())
        return max(0, cache - reserved) + start

    def trim(self) -> None:
        self.stream.synchronize()
        self.b.batch_cache_release()
        self._sg_plans.clear()
        self.torch.cuda.empty_cache()

    def admit(self, req):
        torch = self.torch
        ic = initial_condition(req)
        with torch.cuda.stream(self.copy_stream):
            if req.eq == "nls":
                f0 = torch.from_numpy(ic[0]).pin_memory().to("cuda", self.cdt, non_blocking=True)
                st = {"eq": "nls", "f0": f0, "f1": None, "started": True}
            elif req.eq == "sg":
                u0 = torch.from_numpy(ic[0]).pin_memory().to("cuda", self.rdt, non_blocking=True)
                v0 = torch.from_numpy(ic[1]).pin_memory().to("cuda", self.rdt, non_blocking=True)
                st = {"eq": "sg", "f0": torch.empty_like(u0), "f1": torch.empty_like(u0), "u0": u0, "v0": v0,
                      "started": False}
            else:
                f0 = torch.from_numpy(ic[0]).pin_memory().to("cuda", self.rdt, non_blocking=True)
                st = {"eq": "ns", "f0": f0, "f1": None, "started": True}
            st["ready"] = torch.cuda.Event()
            st["ready"].record(self.copy_stream)
        st["status"] = torch.zeros(1, dtype=torch.int32, device="cuda")
        st["class"] = (req.eq, req.n)
        self._classes[st["class"]] = self._classes.get(st["class"], 0) + 1
        return st

    @property
    def _active_classes(self):
        return [c for c, k in self._classes.items() if k > 0]

    def advance(self, work):
        torch = self.torch
        reqs = []
        with torch.cuda.stream(self.stream):
            for st, k in work:
                self.stream.wait_event(st["ready"])
                if not st["started"]:
                    # the sine-Gordon start-up (u^0, u_t^0) -> (u^0, u^1) counts as step 1
                    plan = self._sg_start_plan(st["f0"].shape[-1])
                    plan.sg_start(st["u0"].unsqueeze(0), st["v0"].unsqueeze(0), st["f0"].unsqueeze(0),
                                  st["f1"].unsqueeze(0), inputs.PAPER_DOMAIN, self.p.sg_dt)
                    st["started"] = True
                    del st["u0"], st["v0"]
                    k -= 1
                if k > 0:
                    reqs.append({"eq": st["eq"], "f0": st["f0"], "f1": st["f1"], "params": self.params[st["eq"]],
                                 "nsteps": k, "dev_status": st["status"]})
            if reqs:
                self.b.solve_batch(reqs, stream=self.stream)
        self.stream.synchronize()

    def _sg_start_plan(self, n):
        key = (n, self.rdt)
        if key not in self._sg_plans:
            prec = self.b.PST_FP64 if self.rdt == self.torch.float64 else self.b.PST_FP32
            self._sg_plans[key] = self.b.Plan(n, n, self.b.PST_R2C, prec, 1, stream=self.stream)
        return self._sg_plans[key]

    def fetch(self, st):
        out = (st["f1"] if st["eq"] == "sg" else st["f0"]).cpu().numpy()
        return out, int(st["status"].item())

    def release(self, st):
        self._classes[st["class"]] -= 1
        st.clear()


def fifo_latencies(requests, service_s: dict) -> dict:
    """Latencies of a single first-in-first-out server that runs each request
    alone for service_s[rid] seconds, with the requests' arrival times: a
    request starts when it has arrived and the previous one has finished
    (the Lindley recursion).  Returns {rid: finish - arrival}."""
    out = {}
    free = 0.0
    for r in sorted(requests, key=lambda r: (r.arrival_s, r.rid)):
        start = max(r.arrival_s, free)
        free = start + service_s[r.rid]
        out[r.rid] = free - r.arrival_s
    return out


def fifo_baseline(requests, params: ServeParams | None = None, fp64: bool = False):
    """The plain path: each request alone, in arrival order, on its own plan
    (the same C-ABI entry points, one simulation per call).  Only the device
    solve of each request is timed (initial conditions and uploads are not).
    Returns (summed solve seconds, pt-steps/s, results by rid, solve seconds
    by rid)."""
    import torch

    from . import binding as b
    p = params or ServeParams()
    rdt, cdt = (torch.float64, torch.complex128) if fp64 else (torch.float32, torch.complex64)
    prec = b.PST_FP64 if fp64 else b.PST_FP32
    plans = {}
    results = {}
    service = {}
    busy = 0.0
    for r in sorted(requests, key=lambda r: r.arrival_s):
        ic = initial_condition(r)
        kind = b.PST_C2C if r.eq == "nls" else b.PST_R2C
        key = (kind, r.n)
        if key not in plans:
            plans[key] = b.Plan(r.n, r.n, kind, prec, 1)
        plan = plans[key]
        if r.eq == "nls":
            f = torch.from_numpy(ic[0]).to("cuda", cdt).unsqueeze(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.nls_step(f, inputs.PAPER_DOMAIN, p.nls_dt, 1.0, r.steps)
            out = f
        elif r.eq == "sg":
            u0 = torch.from_numpy(ic[0]).to("cuda", rdt).unsqueeze(0)
            v0 = torch.from_numpy(ic[1]).to("cuda", rdt).unsqueeze(0)
            a, c = torch.empty_like(u0), torch.empty_like(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.sg_start(u0, v0, a, c, inputs.PAPER_DOMAIN, p.sg_dt)
            plan.sg_step(a, c, inputs.PAPER_DOMAIN, p.sg_dt, r.steps - 1)
            out = c
        else:
            f = torch.from_numpy(ic[0]).to("cuda", rdt).unsqueeze(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.ns_step(f, inputs.NS_DOMAIN, p.ns_dt, p.ns_nu, r.steps, tol=p.ns_tol, max_iter=p.ns_max_iter)
            out = f
        torch.cuda.synchronize()
        service[r.rid] = time.perf_counter() - t0
        busy += service[r.rid]
        results[r.rid] = out[0].cpu().numpy()
    pts = float(sum(r.n * r.n * r.steps for r in requests))
    return busy, pts / busy, results, service
