"""Continuous-batching request loop, driven on the CPU by an executor that
runs the oracle on tiny grids (same interface as the GPU executor)."""
import time

import numpy as np
import pytest

from oracle import nls as onls, ns as ons, sg as osg
from paper_1206_3215_amd import inputs
from paper_1206_3215_amd.serve import BYTES_PER_POINT, Server, ServeParams, fifo_latencies, initial_condition

P = ServeParams()
D = inputs.PAPER_DOMAIN


def solo(req):
    """Oracle result of a request run alone in one go."""
    ic = initial_condition(req)
    if req.eq == "nls":
        return onls.run(ic[0], D.lx, D.ly, P.nls_dt, 1.0, req.steps)[0]
    if req.eq == "sg":
        u1 = osg.start(ic[0], ic[1], D.lx, D.ly, P.sg_dt)
        return osg.run(ic[0], u1, D.lx, D.ly, P.sg_dt, req.steps - 1)[1]
    return ons.run(ic[0], 1.0, 1.0, P.ns_dt, P.ns_nu, req.steps, tol=P.ns_tol, max_iter=P.ns_max_iter)[0]


class OracleExecutor:
    def __init__(self, delay=0.0, fail_rid=None):
        self.delay = delay
        self.fail_rid = fail_rid
        self.in_use = 0
        self.peak = 0
        self.calls = []

    def footprint(self, req):
        return BYTES_PER_POINT[req.eq] * req.n * req.n

    def admit(self, req):
        self.in_use += self.footprint(req)
        self.peak = max(self.peak, self.in_use)
        return {"req": req, "ic": initial_condition(req), "f": None, "g": None, "started": False}

    def advance(self, work):
        self.calls.append([w[0]["req"].rid for w in work])
        time.sleep(self.delay)
        for st, k in work:
            r = st["req"]
            if r.eq == "nls":
                f = st["f"] if st["f"] is not None else st["ic"][0]
                st["f"] = onls.run(f, D.lx, D.ly, P.nls_dt, 1.0, k)[0]
            elif r.eq == "sg":
                if not st["started"]:
                    st["f"], st["g"] = st["ic"][0], osg.start(st["ic"][0], st["ic"][1], D.lx, D.ly, P.sg_dt)
                    st["started"] = True
                    k -= 1
                st["f"], st["g"] = osg.run(st["f"], st["g"], D.lx, D.ly, P.sg_dt, k)
            else:
                f = st["f"] if st["f"] is not None else st["ic"][0]
                st["f"] = ons.run(f, 1.0, 1.0, P.ns_dt, P.ns_nu, k, tol=P.ns_tol, max_iter=P.ns_max_iter)[0]

    def fetch(self, st):
        r = st["req"]
        out = st["g"] if r.eq == "sg" else st["f"]
        return out, (6 if r.rid == self.fail_rid else 0)

    def release(self, st):
        self.in_use -= self.footprint(st["req"])


def small_mix(count=12, rate=200.0):
    return inputs.serving_mix(count, rate_hz=rate, seed=7, log2n_range=(4, 5), steps_range=(3, 11))


def test_results_equal_solo_runs():
    reqs = small_mix()
    rep = Server(OracleExecutor(), budget_bytes=10 ** 9, chunk=4).run(reqs, realtime=False)
    assert [j.req.rid for j in rep.jobs] == [r.rid for r in reqs]
    for j in rep.jobs:
        np.testing.assert_array_equal(j.result, solo(j.req))
    s = rep.summary()
    assert s["requests"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_budget_bounds_resident_footprint():
    reqs = small_mix(16)
    ex = OracleExecutor()
    budget = 3 * BYTES_PER_POINT["sg"] * 32 * 32
    rep = Server(ex, budget_bytes=budget, chunk=3).run(reqs, realtime=False)
    assert len(rep.jobs) == 16 and ex.peak <= budget and ex.in_use == 0


def test_continuous_admission_joins_running_batch():
    # a late arrival is admitted while the first request is still running
    reqs = [inputs.Request(0, "nls", 16, 40, 0.0), inputs.Request(1, "ns", 16, 4, 0.03)]
    ex = OracleExecutor(delay=0.01)
    rep = Server(ex, budget_bytes=10 ** 9, chunk=2).run(reqs, realtime=True)
    j0, j1 = rep.jobs
    assert j1.t_admit < j0.t_done
    assert any(set(c) == {0, 1} for c in ex.calls)      # shared chunks
    for j in rep.jobs:
        np.testing.assert_array_equal(j.result, solo(j.req))


def test_failure_is_isolated():
    reqs = small_mix(6)
    rep = Server(OracleExecutor(fail_rid=2), budget_bytes=10 ** 9, chunk=5).run(reqs, realtime=False)
    for j in rep.jobs:
        assert j.status == (6 if j.req.rid == 2 else 0)
        np.testing.assert_array_equal(j.result, solo(j.req))


def test_request_larger_than_budget_rejected():
    with pytest.raises(ValueError):
        Server(OracleExecutor(), budget_bytes=100).run([inputs.Request(0, "nls", 16, 3, 0.0)])


class ChunkStatusExecutor(OracleExecutor):
    """Reports NOT_CONVERGED for one request on its first chunk only (the
    per-chunk statuses a device executor would return), OK at fetch."""

    def __init__(self, rid):
        super().__init__()
        self.rid = rid
        self.reported = False

    def advance(self, work):
        super().advance(work)
        out = []
        for st, _ in work:
            hit = st["req"].rid == self.rid and not self.reported
            self.reported = self.reported or hit
            out.append(5 if hit else 0)
        return out

    def fetch(self, st):
        return super().fetch(st)[0], 0


def test_status_is_latched_over_chunks():
    reqs = small_mix(6)
    rid = max(reqs, key=lambda r: r.steps).rid          # runs for several chunks
    rep = Server(ChunkStatusExecutor(rid), budget_bytes=10 ** 9, chunk=2).run(reqs, realtime=False)
    for j in rep.jobs:
        assert j.status == (5 if j.req.rid == rid else 0)


class OverheadExecutor(OracleExecutor):
    """Holds device memory beyond the reservations (a library cache) that
    only trim() gives back."""

    def __init__(self, extra):
        super().__init__()
        self.extra = extra
        self.trims = 0
        self.peak_total = 0

    def admit(self, req):
        st = super().admit(req)
        self.peak_total = max(self.peak_total, self.in_use + self.extra)
        return st

    def overhead_bytes(self):
        return self.extra

    def trim(self):
        self.trims += 1
        self.extra = 0


def test_executor_overhead_counts_against_budget():
    reqs = small_mix(10)
    budget = 4 * BYTES_PER_POINT["sg"] * 32 * 32
    ex = OverheadExecutor(extra=budget // 2)
    rep = Server(ex, budget_bytes=budget, chunk=3).run(reqs, realtime=False)
    assert len(rep.jobs) == 10 and ex.peak_total <= budget
    assert ex.trims >= 1                                 # released when admission was blocked
    for j in rep.jobs:
        np.testing.assert_array_equal(j.result, solo(j.req))


def test_fifo_latencies_follow_the_single_server_queue():
    # arrivals 0, 1, 1.5, 10 with solve times 2, 1, 0.5, 1: starts 0, 2, 3, 10 (the server is
    # idle from 3.5 to 10), finishes 2, 3, 3.5, 11
    reqs = [inputs.Request(rid=i, eq="nls", n=8, steps=1, arrival_s=a)
            for i, a in enumerate([0.0, 1.0, 1.5, 10.0])]
    lat = fifo_latencies(reqs[::-1], {0: 2.0, 1: 1.0, 2: 0.5, 3: 1.0})
    assert lat == pytest.approx({0: 2.0, 1: 2.0, 2: 2.0, 3: 1.0})


class StepRecorder(OracleExecutor):
    def __init__(self):
        super().__init__(delay=0.005)
        self.steps = []

    def advance(self, work):
        self.steps.append({st["req"].rid: k for st, k in work})
        return super().advance(work)


def test_age_weighted_chunks_grow_with_waiting_and_keep_results():
    # with age_s far below a round's duration, a request that has waited
    # advances by several chunks per round (capped by max_boost and by its
    # remaining steps); the results stay those of solo runs
    reqs = [inputs.Request(0, "nls", 16, 30, 0.0), inputs.Request(1, "sg", 16, 9, 0.0),
            inputs.Request(2, "ns", 16, 5, 0.0)]
    ex = StepRecorder()
    rep = Server(ex, budget_bytes=10 ** 9, chunk=2, age_s=1e-4, max_boost=4).run(reqs, realtime=True)
    assert max(k for call in ex.steps for k in call.values()) == 8      # chunk x max_boost
    assert all(k <= 8 for call in ex.steps for k in call.values())
    assert sum(call.get(0, 0) for call in ex.steps) == 30
    for j in rep.jobs:
        np.testing.assert_array_equal(j.result, solo(j.req))
