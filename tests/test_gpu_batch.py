"""solve_batch: mixed equations and uneven sizes in one call vs the single-plan path."""
import numpy as np
import pytest

from paper_1206_3215_amd import inputs
from tests.gpuutil import need_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
D_NLS, D_SG, D_NS = inputs.PAPER_DOMAIN, inputs.PAPER_DOMAIN, inputs.NS_DOMAIN


def single(eq, f0, f1, prm, nsteps, prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    ny, nx = f0.shape
    kind = b.PST_C2C if eq == "nls" else b.PST_R2C
    plan = b.Plan(nx, ny, kind, prec, 1)
    dt = plan.complex_dtype if eq == "nls" else plan.real_dtype
    a = to_dev(f0[None], torch, dt)
    if eq == "nls":
        plan.nls_step(a, D_NLS, prm["dt"], 1.0, nsteps)
        return to_host(a)[0], None
    if eq == "sg":
        bb = to_dev(f1[None], torch, dt)
        plan.sg_step(a, bb, D_SG, prm["dt"], nsteps)
        return to_host(a)[0], to_host(bb)[0]
    plan.ns_step(a, D_NS, prm["dt"], prm["nu"], nsteps, tol=prm.get("tol", 1e-10),
                 max_iter=prm.get("max_iter", 50), fixed_iters=prm.get("fixed", 0))
    return to_host(a)[0], None


def build_mix(prec):
    rng = np.random.default_rng(0)
    mix = []
    for i, (n, steps) in enumerate([(64, 7), (64, 7), (64, 3), (128, 5)]):
        mix.append(("nls", inputs.nls_gaussian(n, n, D_NLS, seed=i), None, {"dt": 1e-3}, steps))
    for i, (nx, ny) in enumerate([(32, 64), (32, 64), (128, 128)]):
        u0, _ = inputs.sg_gaussian(nx, ny, D_SG, seed=i)
        mix.append(("sg", u0 - 0.01 * rng.standard_normal(u0.shape), u0, {"dt": 0.01}, 6))
    for i, n in enumerate([64, 64, 128]):
        mix.append(("ns", inputs.ns_random_phase(n, seed=i), None, {"dt": 1e-3, "nu": 1e-3, "fixed": 2}, 4))
    mix.append(("ns", inputs.ns_random_phase(64, seed=9), None, {"dt": 1e-3, "nu": 1e-3}, 3))
    return mix


def oracle_run(eq, f0, f1, prm, nsteps):
    """The request's result computed by the FP64 oracle."""
    from oracle import nls as onls, ns as ons, sg as osg
    if eq == "nls":
        return onls.run(f0, D_NLS.lx, D_NLS.ly, prm["dt"], 1.0, nsteps)[0], None
    if eq == "sg":
        a, c = osg.run(f0, f1, D_SG.lx, D_SG.ly, prm["dt"], nsteps)
        return a, c
    return ons.run(f0, D_NS.lx, D_NS.ly, prm["dt"], prm["nu"], nsteps, tol=prm.get("tol", 1e-10),
                   max_iter=prm.get("max_iter", 50), fixed_iters=prm.get("fixed", 0))[0], None


@pytest.mark.parametrize("prec", [1, 0])
def test_mixed_batch_matches_single_runs(prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    mix = build_mix(prec)
    reqs, tens = [], []
    for eq, f0, f1, prm, steps in mix:
        cdt = (torch.complex128 if prec else torch.complex64) if eq == "nls" else (torch.float64 if prec else torch.float32)
        a = to_dev(f0, torch, cdt)
        bb = to_dev(f1, torch, cdt) if f1 is not None else None
        d = {"nls": D_NLS, "sg": D_SG, "ns": D_NS}[eq]
        pr = b.make_params(eq, d, prm["dt"], nu=prm.get("nu", 0.0), fixed_iters=prm.get("fixed", 0))
        reqs.append({"eq": eq, "f0": a, "f1": bb, "params": pr, "nsteps": steps,
                     "dev_status": torch.full((1,), -1, dtype=torch.int32, device="cuda")})
        tens.append((a, bb))
    b.solve_batch(reqs)
    torch.cuda.synchronize()
    tol = 1e-11 if prec else 1e-4
    for (eq, f0, f1, prm, steps), (a, bb), r in zip(mix, tens, reqs):
        ref0, ref1 = single(eq, f0, f1, prm, steps, prec)
        assert rel_err(to_host(a), ref0) < tol, (eq, f0.shape, steps)
        if ref1 is not None:
            assert rel_err(to_host(bb), ref1) < tol
        assert int(r["dev_status"].item()) == 0
        # and against the oracle directly (SG: f0, f1 = u_prev, u_curr)
        o0, o1 = oracle_run(eq, f0, f1, prm, steps)
        assert rel_err(to_host(a), o0) < tol, ("oracle", eq, f0.shape, steps)
        if o1 is not None:
            assert rel_err(to_host(bb), o1) < tol, ("oracle", eq, f0.shape, steps)


def test_uneven_ns_batch_bitwise_vs_alone():
    # 4 x 1024^2 + 4 x 2048^2 vorticity fields, fixed iterations, FP32
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    fields = [inputs.ns_random_phase(1024 if s < 4 else 2048, seed=s) for s in range(8)]
    pr = b.make_params("ns", D_NS, 1e-3, nu=1e-3, fixed_iters=2)
    ts = [to_dev(f, torch, torch.float32) for f in fields]
    b.solve_batch([{"eq": "ns", "f0": t, "params": pr, "nsteps": 3} for t in ts])
    alone = to_dev(fields[5], torch, torch.float32)
    b.solve_batch([{"eq": "ns", "f0": alone, "params": pr, "nsteps": 3}])
    torch.cuda.synchronize()
    assert np.array_equal(to_host(alone), to_host(ts[5]))
    ref, _ = single("ns", fields[1], None, {"dt": 1e-3, "nu": 1e-3, "fixed": 2}, 3, 0)
    assert np.array_equal(to_host(ts[1]), ref)


def test_adaptive_ns_group_larger_than_the_first_on_a_cached_plan():
    # A group of 3 sizes an internal plan for 4 fields; a later group of 4 of
    # the same class runs on that plan, with more convergence flags to copy
    # back each step than the first group had.
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    fields = [inputs.ns_random_phase(64, seed=s) for s in range(4)]
    pr = b.make_params("ns", D_NS, 1e-3, nu=1e-3, tol=1e-10)
    first = [to_dev(f, torch, torch.float64) for f in fields[:3]]
    b.solve_batch([{"eq": "ns", "f0": t, "params": pr, "nsteps": 2} for t in first])
    ts = [to_dev(f, torch, torch.float64) for f in fields]
    st = [torch.full((1,), -1, dtype=torch.int32, device="cuda") for _ in ts]
    b.solve_batch([{"eq": "ns", "f0": t, "params": pr, "nsteps": 2, "dev_status": s} for t, s in zip(ts, st)])
    torch.cuda.synchronize()
    assert all(int(s.item()) == 0 for s in st)
    for i in (0, 3):
        ref, _ = single("ns", fields[i], None, {"dt": 1e-3, "nu": 1e-3, "tol": 1e-10}, 2, 1)
        assert rel_err(to_host(ts[i]), ref) < 1e-12, i


def test_repeat_call_replays_graph_and_matches_double_steps():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    f = [inputs.nls_gaussian(128, 128, D_NLS, seed=s) for s in range(3)]
    ts = [to_dev(x, torch, torch.complex128) for x in f]
    pr = b.make_params("nls", D_NLS, 1e-3)
    for _ in range(3):
        b.solve_batch([{"eq": "nls", "f0": t, "params": pr, "nsteps": 5} for t in ts])
    torch.cuda.synchronize()
    plan = b.Plan(128, 128, b.PST_C2C, b.PST_FP64, 1)
    a = to_dev(f[2][None], torch, torch.complex128)
    for _ in range(3):
        plan.nls_step(a, D_NLS, 1e-3, 1.0, 5)
    assert np.array_equal(to_host(a)[0], to_host(ts[2]))


def test_not_converged_status_is_per_request():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    good = b.make_params("ns", D_NS, 1e-3, nu=1e-3, tol=1e-10, max_iter=50)
    bad = b.make_params("ns", D_NS, 1e-3, nu=1e-3, tol=0.0, max_iter=2)
    ts = [to_dev(inputs.ns_random_phase(32, seed=s), torch, torch.float64) for s in range(2)]
    st = [torch.full((1,), -1, dtype=torch.int32, device="cuda") for _ in range(2)]
    b.solve_batch([{"eq": "ns", "f0": ts[0], "params": good, "nsteps": 2, "dev_status": st[0]},
                   {"eq": "ns", "f0": ts[1], "params": bad, "nsteps": 2, "dev_status": st[1]}])
    torch.cuda.synchronize()
    assert int(st[0].item()) == b.PST_OK and int(st[1].item()) == b.PST_ERR_NOT_CONVERGED


def test_invalid_requests_rejected_on_host():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    t = to_dev(np.zeros((48, 48)), torch, torch.float32)
    with pytest.raises(b.PstError):
        b.solve_batch([{"eq": "ns", "f0": t, "params": b.make_params("ns", D_NS, 1e-3), "nsteps": 1}])


def test_params_change_between_calls_is_not_replayed_stale():
    # Three calls on the same tensors and schedule capture and replay a graph;
    # three more with another time step (no host sync between any of them)
    # must run with the new step: the replay key includes the parameters, and
    # the propagator tables are rewritten only after the old steps finished.
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    f = [inputs.nls_gaussian(128, 128, D_NLS, seed=s) for s in range(3)]
    u = [inputs.sg_gaussian(64, 64, D_SG, seed=s)[0] for s in range(2)]
    ts = [to_dev(x, torch, torch.complex128) for x in f]
    ua = [to_dev(x, torch, torch.float64) for x in u]
    ub = [to_dev(x * 1.01, torch, torch.float64) for x in u]
    for dt_nls, dt_sg in ((1e-3, 0.01), (3e-3, 0.02)):
        pn, ps = b.make_params("nls", D_NLS, dt_nls), b.make_params("sg", D_SG, dt_sg)
        for _ in range(3):
            b.solve_batch([{"eq": "nls", "f0": t, "params": pn, "nsteps": 5} for t in ts]
                          + [{"eq": "sg", "f0": x, "f1": y, "params": ps, "nsteps": 4} for x, y in zip(ua, ub)])
    torch.cuda.synchronize()
    plan = b.Plan(128, 128, b.PST_C2C, b.PST_FP64, 1)
    a = to_dev(f[1][None], torch, torch.complex128)
    sp = b.Plan(64, 64, b.PST_R2C, b.PST_FP64, 1)
    x, y = to_dev(u[1][None], torch, torch.float64), to_dev(u[1][None] * 1.01, torch, torch.float64)
    for dt_nls, dt_sg in ((1e-3, 0.01), (3e-3, 0.02)):
        for _ in range(3):
            plan.nls_step(a, D_NLS, dt_nls, 1.0, 5)
            sp.sg_step(x, y, D_SG, dt_sg, 4)
    assert np.array_equal(to_host(a)[0], to_host(ts[1]))
    assert np.array_equal(to_host(x)[0], to_host(ua[1])) and np.array_equal(to_host(y)[0], to_host(ub[1]))


def _requests_with_one_nan(torch, b, prec):
    """A mixed call: NLS, SG, NS fixed-iteration and NS adaptive groups, each
    with one request whose initial field holds a NaN."""
    cdt = torch.complex128 if prec else torch.complex64
    rdt = torch.float64 if prec else torch.float32
    pn = b.make_params("nls", D_NLS, 1e-3)
    ps = b.make_params("sg", D_SG, 0.01)
    pf = b.make_params("ns", D_NS, 1e-3, nu=1e-3, fixed_iters=2)
    pa = b.make_params("ns", D_NS, 1e-3, nu=1e-3, tol=1e-10)
    reqs = []
    for i in range(3):
        reqs.append({"eq": "nls", "f0": to_dev(inputs.nls_gaussian(64, 64, D_NLS, seed=i), torch, cdt),
                     "params": pn, "nsteps": 6})
    for i in range(2):
        u0 = inputs.sg_gaussian(64, 64, D_SG, seed=i)[0]
        reqs.append({"eq": "sg", "f0": to_dev(u0, torch, rdt), "f1": to_dev(u0 * 0.99, torch, rdt),
                     "params": ps, "nsteps": 5})
    for pr in (pf, pa):
        for i in range(2):
            reqs.append({"eq": "ns", "f0": to_dev(inputs.ns_random_phase(32, seed=i), torch, rdt),
                         "params": pr, "nsteps": 3})
    bad = [1, 4, 5, 8]
    for i in bad:
        reqs[i]["f0"].view(-1)[7] = float("nan")
    for r in reqs:
        r["dev_status"] = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    return reqs, bad


@pytest.mark.parametrize("prec", [1, 0])
def test_nonfinite_request_is_reported_and_isolated(prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    reqs, bad = _requests_with_one_nan(torch, b, prec)
    alone, _ = _requests_with_one_nan(torch, b, prec)
    b.solve_batch(reqs)
    for r in alone:
        b.solve_batch([r])
    torch.cuda.synchronize()
    for i, (r, a) in enumerate(zip(reqs, alone)):
        st = int(r["dev_status"].item())
        assert st == (b.PST_ERR_NONFINITE if i in bad else b.PST_OK), (i, r["eq"], st)
        assert int(a["dev_status"].item()) == st
        if i not in bad:
            assert np.array_equal(to_host(r["f0"]), to_host(a["f0"])), (i, r["eq"])


def test_status_latches_across_calls():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    bad = b.make_params("ns", D_NS, 1e-3, nu=1e-3, tol=0.0, max_iter=2)
    good = b.make_params("ns", D_NS, 1e-3, nu=1e-3, tol=1e-10, max_iter=50)
    w = to_dev(inputs.ns_random_phase(32, seed=0), torch, torch.float64)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.solve_batch([{"eq": "ns", "f0": w, "params": bad, "nsteps": 1, "dev_status": st}])
    b.solve_batch([{"eq": "ns", "f0": w, "params": good, "nsteps": 2, "dev_status": st}])
    torch.cuda.synchronize()
    assert int(st.item()) == b.PST_ERR_NOT_CONVERGED
    st.zero_()
    b.solve_batch([{"eq": "ns", "f0": w, "params": good, "nsteps": 2, "dev_status": st}])
    torch.cuda.synchronize()
    assert int(st.item()) == b.PST_OK


def test_nonfinite_latched_for_single_plan_entry_points():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    plan = b.Plan(64, 64, b.PST_C2C, b.PST_FP32, 2)
    psi = to_dev(np.stack([inputs.nls_gaussian(64, 64, D_NLS, seed=s) for s in range(2)]), torch,
                 torch.complex64)
    plan.nls_step(psi, D_NLS, 1e-3, 1.0, 3)
    assert plan.sync_status() == b.PST_OK
    psi[1, 5, 5] = float("inf")
    plan.nls_step(psi, D_NLS, 1e-3, 1.0, 3)
    assert plan.sync_status() == b.PST_ERR_NONFINITE
    assert plan.sync_status() == b.PST_OK                 # read clears it
    sp = b.Plan(64, 64, b.PST_R2C, b.PST_FP64, 1)
    u = to_dev(inputs.sg_gaussian(64, 64, D_SG, seed=0)[0][None], torch, torch.float64)
    v = u.clone()
    v[0, 3, 3] = float("nan")
    sp.sg_step(u, v, D_SG, 0.01, 2)
    assert sp.sync_status() == b.PST_ERR_NONFINITE


def test_misaligned_fields_rejected():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    buf = torch.zeros(64 * 64 + 1, dtype=torch.complex128, device="cuda")
    off = buf[1:].view(64, 64)                            # 16 bytes past a 256-byte boundary
    assert off.data_ptr() % 256 != 0
    with pytest.raises(b.PstError, match="aligned"):
        b.solve_batch([{"eq": "nls", "f0": off, "params": b.make_params("nls", D_NLS, 1e-3), "nsteps": 1}])
    plan = b.Plan(64, 64, b.PST_C2C, b.PST_FP64, 1)
    with pytest.raises(b.PstError, match="aligned"):
        plan.nls_step(off.view(1, 64, 64), D_NLS, 1e-3, 1.0, 1)
