"""Navier-Stokes (CN + fixed point) through the C ABI vs the FP64 oracle."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ns as ons
from paper_1206_3215_amd import inputs
from tests.gpuutil import need_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = {0: 1e-4, 1: 1e-11}
D1 = inputs.NS_DOMAIN


def gpu_ns(w0, d, dt, nu, nsteps, prec, tol=1e-10, max_iter=50, fixed=0, want_iters=False, variant=0):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    w0 = w0 if w0.ndim == 3 else w0[None]
    batch, ny, nx = w0.shape
    plan = b.Plan(nx, ny, b.PST_R2C, prec, batch)
    plan.set_column_variant(variant)
    W = to_dev(w0, torch, plan.real_dtype)
    its = torch.zeros(max(nsteps, 1) * batch, dtype=torch.int32, device="cuda")
    plan.ns_step(W, d, dt, nu, nsteps, tol=tol, max_iter=max_iter, fixed_iters=fixed,
                 dev_iters=its if want_iters else None)
    st = plan.sync_status()
    return to_host(W), to_host(its).reshape(-1, batch), st, plan


@pytest.mark.parametrize("n", [64, 128])
def test_paper_table4_worked_example_on_gpu(golden_dir, n):
    # Table 4: 20 steps of dt 1.25e-3, tol 1e-10, max error 1.65e-5 vs Taylor-Green (nu = 0.1)
    g = json.load(open(os.path.join(golden_dir, "paper_table4_taylor_green.json")))
    nu = 0.1
    w, its, st, _ = gpu_ns(inputs.taylor_green(n, 0.0, nu), D1, g["dt"], nu, g["steps"], 1, tol=g["tol"],
                           want_iters=True)
    assert st == 0
    err = np.max(np.abs(w[0] - inputs.taylor_green(n, g["steps"] * g["dt"], nu)))
    assert abs(err - g["max_error"]) < 0.005e-5
    ref, rits, _ = ons.run(inputs.taylor_green(n, 0.0, nu), 1.0, 1.0, g["dt"], nu, g["steps"], tol=g["tol"])
    assert rel_err(w[0], ref) < TOL[1]
    assert list(its[:, 0]) == rits


@pytest.mark.parametrize("prec", [1, 0])
def test_taylor_green_cn_ratio_large_grid(prec):
    n, dt, nu, steps = 1024, 1e-3, 1e-3, 50
    w, _, st, _ = gpu_ns(inputs.taylor_green(n), D1, dt, nu, steps, prec, fixed=2)
    k2 = 8 * math.pi ** 2
    rho = (1 - 0.5 * dt * nu * k2) / (1 + 0.5 * dt * nu * k2)
    assert rel_err(w[0], rho ** steps * inputs.taylor_green(n)) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("n,batch", [(32, 1), (64, 3), (128, 1)])
def test_random_phase_fixed_iterations(n, batch, prec):
    w0 = np.stack([inputs.ns_random_phase(n, seed=s) for s in range(batch)])
    got, _, st, _ = gpu_ns(w0, D1, 1e-3, 1e-3, 10, prec, fixed=3)
    for i in range(batch):
        ref, _, _ = ons.run(w0[i], 1.0, 1.0, 1e-3, 1e-3, 10, fixed_iters=3)
        assert rel_err(got[i], ref) < TOL[prec], i


def test_non_square_domain_and_grid():
    d = inputs.Domain(2.0, 1.0, 0.0, 0.0)
    rng = np.random.default_rng(4)
    w0 = np.fft.irfft2(np.where(np.random.default_rng(1).random((16, 17)) < 0.3,
                                rng.standard_normal((16, 17)) + 1j * rng.standard_normal((16, 17)), 0), s=(16, 32))
    w0 *= 5 / np.max(np.abs(w0))
    got, _, _, _ = gpu_ns(w0, d, 2e-3, 1e-2, 6, 1, fixed=2)
    ref, _, _ = ons.run(w0, d.lx, d.ly, 2e-3, 1e-2, 6, fixed_iters=2)
    assert rel_err(got[0], ref) < TOL[1]


def test_adaptive_with_nyquist_content_matches_oracle():
    # Content in the x-Nyquist column (not truncated by the initial field):
    # after a step's first iteration it is left out of the column pass, its
    # stored residual term must then not count.  Iteration counts and the
    # field must still match the oracle's adaptive run.
    n = 32
    rng = np.random.default_rng(7)
    spec = rng.standard_normal((n, n // 2 + 1)) + 1j * rng.standard_normal((n, n // 2 + 1))
    w0 = np.fft.irfft2(spec, s=(n, n))
    w0 *= 20 / np.max(np.abs(w0))
    assert np.max(np.abs(np.fft.rfft2(w0)[:, n // 2])) > 1.0
    got, its, st, _ = gpu_ns(w0, D1, 1e-3, 1e-2, 6, 1, tol=1e-10, want_iters=True)
    ref, rits, ok = ons.run(w0, 1.0, 1.0, 1e-3, 1e-2, 6, tol=1e-10)
    assert ok and st == 0
    assert list(its[:, 0]) == rits
    assert rel_err(got[0], ref) < TOL[1]


def test_adaptive_iterations_match_oracle():
    w0 = inputs.ns_random_phase(64, seed=3)
    got, its, st, _ = gpu_ns(w0, D1, 1e-3, 1e-3, 8, 1, tol=1e-10, want_iters=True)
    ref, rits, ok = ons.run(w0, 1.0, 1.0, 1e-3, 1e-3, 8, tol=1e-10)
    assert ok and st == 0
    assert list(its[:, 0]) == rits
    assert rel_err(got[0], ref) < TOL[1]


def test_not_converged_is_latched_from_host_side_limit():
    from paper_1206_3215_amd import binding as b
    w0 = inputs.ns_random_phase(32, seed=1)
    got, its, st, _ = gpu_ns(w0, D1, 1e-3, 1e-3, 1, 1, tol=0.0, max_iter=3, want_iters=True)
    assert st == b.PST_ERR_NOT_CONVERGED
    assert its[0, 0] == 3
    ref, rits, ok = ons.run(w0, 1.0, 1.0, 1e-3, 1e-3, 1, tol=0.0, max_iter=3)
    assert not ok and rits == [3] and rel_err(got[0], ref) < TOL[1]


@pytest.mark.parametrize("prec", [1, 0])
def test_energy_enstrophy(prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    w0 = np.stack([inputs.taylor_green(64), inputs.ns_random_phase(64, seed=2)])
    plan = b.Plan(64, 64, b.PST_R2C, prec, 2)
    q = plan.conserved_quantities("ns", to_dev(w0, torch, plan.real_dtype), d=D1)
    tq = 1e-12 if prec else 1e-6
    assert abs(q[0, 0] - 0.25) < tq and abs(q[0, 1] / (2 * math.pi ** 2) - 1) < tq
    assert abs(q[1, 0] / ons.energy(w0[1], 1, 1) - 1) < tq
    assert abs(q[1, 1] / ons.enstrophy(w0[1], 1, 1) - 1) < tq


@pytest.mark.parametrize("n,variant", [(1024, v) for v in range(4)] + [(2048, v) for v in range(4)])
def test_full_size_random_phase_short(n, variant):
    # benchmark grids (uneven batch members) in both column variants, FP32,
    # fixed 2 iterations, 4 steps
    w0 = inputs.ns_random_phase(n, seed=4)
    got, _, _, _ = gpu_ns(w0, D1, 1e-3, 1e-3, 4, 0, fixed=2, variant=variant)
    ref, _, _ = ons.run(w0, 1.0, 1.0, 1e-3, 1e-3, 4, fixed_iters=2)
    assert rel_err(got[0], ref) < TOL[0]


@pytest.mark.parametrize("n", [1024, 2048])
def test_full_size_random_phase_adaptive_converges(n):
    # the benchmark configuration (FP32, tol 1e-10, dt 2.5e-4): every step
    # converges in a few iterations and the field stays finite; the first
    # step agrees with the FP64 oracle's adaptive step
    w0 = inputs.ns_random_phase(n, seed=5)
    got, its, st, _ = gpu_ns(w0, D1, 2.5e-4, 1e-3, 3, 0, tol=1e-10, max_iter=50, want_iters=True)
    assert st == 0
    assert np.all(np.isfinite(got)) and np.all((its >= 2) & (its <= 12))
    one, _, _, _ = gpu_ns(w0, D1, 2.5e-4, 1e-3, 1, 0, tol=1e-10, max_iter=50)
    ref, _, ok = ons.run(w0, 1.0, 1.0, 2.5e-4, 1e-3, 1, tol=1e-10, max_iter=50)
    assert ok and rel_err(one[0], ref) < TOL[0]


def test_batch_member_bitwise_equal_alone():
    w0 = np.stack([inputs.ns_random_phase(128, seed=s) for s in range(4)])
    got, _, _, _ = gpu_ns(w0, D1, 1e-3, 1e-3, 5, 0, tol=1e-10)
    alone, _, _, _ = gpu_ns(w0[2:3], D1, 1e-3, 1e-3, 5, 0, tol=1e-10)
    assert np.array_equal(got[2], alone[0])


def test_parked_field_resumes_and_matches_oracle():
    # Iterations are queued ahead of the host (the predicted count plus one);
    # a field that needs more is parked and resumed by the host.  Here one
    # field needs 6 iterations per step and the others fewer: the first call
    # (prediction 3) parks the hard field on its first step while the others
    # finish the chunk; the second call on the same plan (prediction 6)
    # parks nothing.  Every field and every step's iteration count must
    # match the oracle's adaptive run.
    hard = inputs.ns_random_phase(64, seed=3)
    easy = [0.05 * inputs.ns_random_phase(64, seed=s) for s in (4, 5)]
    w0 = np.stack([easy[0], hard, easy[1]])
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    plan = b.Plan(64, 64, b.PST_R2C, b.PST_FP64, 3)
    W = to_dev(w0, torch, torch.float64)
    for call in range(2):
        its = torch.zeros(5 * 3, dtype=torch.int32, device="cuda")
        before = to_host(W).copy()
        plan.ns_step(W, D1, 1e-3, 1e-3, 5, tol=1e-10, dev_iters=its)
        assert plan.sync_status() == b.PST_OK
        got, its = to_host(W), to_host(its).reshape(5, 3)
        for i in range(3):
            ref, rits, ok = ons.run(before[i], 1.0, 1.0, 1e-3, 1e-3, 5, tol=1e-10)
            assert ok and list(its[:, i]) == rits, (call, i, its[:, i], rits)
            assert rel_err(got[i], ref) < TOL[1], (call, i)
        assert max(its[:, 1]) > 4 > max(its[:, 0])       # the hard field outran the first prediction


def test_fixed_iterations_need_no_host_wait_and_match_adaptive_counts():
    # fixed-K mode queues exactly K iterations per step (no parking); with K
    # equal to the adaptive count the two agree to rounding
    w0 = inputs.ns_random_phase(64, seed=3)
    fixed, _, st, _ = gpu_ns(w0, D1, 1e-3, 1e-3, 4, 1, fixed=6)
    adapt, its, _, _ = gpu_ns(w0, D1, 1e-3, 1e-3, 4, 1, tol=1e-10, want_iters=True)
    assert st == 0 and list(its[:, 0]) == [6, 6, 6, 6]
    assert rel_err(fixed[0], adapt[0]) < 1e-13
