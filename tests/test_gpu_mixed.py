"""Grids whose sides are 2^a 3^b 5^c but not powers of two (mixed-radix
passes) through the C ABI: 2D transforms against the oracle's FFT, the NLS
split step against the plane-wave closed form and the oracle, its
diagnostics, batched requests, and the equations that stay power-of-two
only."""
import math

import numpy as np
import pytest

from oracle import nls as onls
from oracle import spectral as sp
from paper_1206_3215_amd import inputs
from tests.gpuutil import need_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = {0: 1e-4, 1: 1e-11}
FTOL = {0: 1e-5, 1: 1e-13}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nx,ny,batch", [(12, 20, 2), (15, 9, 1), (96, 96, 1), (1536, 96, 1), (24, 3000, 1),
                                         (1536, 1536, 1), (3000, 3000, 1), (6, 4096, 1), (4800, 12, 1)])
def test_c2c_against_oracle(nx, ny, batch, prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    rng = np.random.default_rng(nx + 7 * ny)
    x = rng.standard_normal((batch, ny, nx)) + 1j * rng.standard_normal((batch, ny, nx))
    plan = b.Plan(nx, ny, b.PST_C2C, prec, batch)
    xd = to_dev(x, torch, plan.complex_dtype)
    yd = torch.empty_like(xd)
    plan.fft2d_exec(xd, yd, -1)
    ref = np.stack([sp.fft2(x[i]) for i in range(batch)])
    bar = FTOL[prec] * math.log2(nx * ny)
    assert rel_err(to_host(yd), ref) < bar
    plan.fft2d_exec(yd, yd, +1)
    assert rel_err(to_host(yd), x) < bar


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nx,ny,batch", [(12, 20, 3), (15, 9, 1), (96, 96, 1), (1536, 1536, 1), (3000, 24, 1)])
def test_r2c_c2r_against_oracle(nx, ny, batch, prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    rng = np.random.default_rng(3 * nx + ny)
    x = rng.standard_normal((batch, ny, nx))
    plan = b.Plan(nx, ny, b.PST_R2C, prec, batch)
    xd = to_dev(x, torch, plan.real_dtype)
    yd = torch.empty((batch, ny, nx // 2 + 1), dtype=plan.complex_dtype, device="cuda")
    plan.fft2d_exec(xd, yd, -1)
    ref = np.stack([sp.rfft2(x[i]) for i in range(batch)])
    bar = FTOL[prec] * math.log2(nx * ny)
    assert rel_err(to_host(yd), ref) < bar
    zd = torch.empty_like(xd)
    plan.fft2d_exec(yd, zd, +1)
    assert rel_err(to_host(zd), x) < bar


def run_nls(psi0, d, dt, g, nsteps, prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    batch = psi0.shape[0] if psi0.ndim == 3 else 1
    ny, nx = psi0.shape[-2:]
    plan = b.Plan(nx, ny, b.PST_C2C, prec, batch)
    plan.autotune("nls")                       # one configuration: a no-op
    psi = to_dev(psi0.reshape(batch, ny, nx), torch, plan.complex_dtype)
    q0 = plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g)
    plan.nls_step(psi, d, dt, g, nsteps)
    q1 = plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g)
    assert plan.sync_status() == b.PST_OK
    return to_host(psi).reshape(psi0.shape), q0, q1


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("n", [96, 1536, 3000])
def test_nls_plane_wave_closed_form(n, prec):
    # psi = A exp(i(k.x - (|k|^2 + g|A|^2) t)) is reproduced exactly by the
    # split step for any dt, on any grid
    L, A, dt, steps = 10 * math.pi, 0.3, 1e-3, 30
    X, Y = inputs.grid(n, n, inputs.Domain(L, L, 0, 0))
    k = 2 * math.pi * np.array([7, -3]) / L
    psi0 = A * np.exp(1j * (k[0] * X + k[1] * Y))
    got, q0, q1 = run_nls(psi0, inputs.Domain(L, L, 0, 0), dt, 1.0, steps, prec)
    exact = psi0 * np.exp(-1j * (k @ k + A * A) * dt * steps)
    assert rel_err(got, exact) < TOL[prec]
    # mass |A|^2 L^2 and energy (|k|^2 |A|^2/2 + |A|^4/4) L^2 of the plane wave
    assert abs(q0[0, 0] / (A * A * L * L) - 1) < TOL[prec]
    assert abs(q0[0, 1] / ((0.5 * (k @ k) * A * A + 0.25 * A ** 4) * L * L) - 1) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("nx,ny,batch", [(96, 96, 1), (120, 40, 2), (1536, 1536, 1), (15, 25, 1)])
def test_nls_gaussian_against_oracle(nx, ny, batch, prec):
    d = inputs.PAPER_DOMAIN
    psi0 = np.stack([inputs.nls_gaussian(nx, ny, d, seed=s) for s in range(batch)])
    got, q0, q1 = run_nls(psi0, d, 1e-3, 1.0, 10, prec)
    for i in range(batch):
        ref, diag = onls.run(psi0[i], d.lx, d.ly, 1e-3, 1.0, 10, diag_every=10)
        assert rel_err(got[i], ref) < TOL[prec]
        for q, (_, m, e) in ((q0, diag[0]), (q1, diag[1])):
            assert abs(q[i, 0] / m - 1) < (1e-12 if prec else 1e-5)
            assert abs(q[i, 1] / e - 1) < (1e-12 if prec else 1e-5)


def test_batched_requests_of_mixed_sizes_against_oracle():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    d = inputs.PAPER_DOMAIN
    sizes = [(96, 96), (96, 96), (160, 60), (128, 128)]
    psi0 = [inputs.nls_gaussian(nx, ny, d, seed=i) for i, (nx, ny) in enumerate(sizes)]
    ts = [to_dev(p, torch, torch.complex128) for p in psi0]
    st = [torch.full((1,), -1, dtype=torch.int32, device="cuda") for _ in ts]
    pr = b.make_params("nls", d, 1e-3)
    b.solve_batch([{"eq": "nls", "f0": t, "params": pr, "nsteps": 6, "dev_status": s} for t, s in zip(ts, st)])
    torch.cuda.synchronize()
    for p, t, s in zip(psi0, ts, st):
        ref, _ = onls.run(p, d.lx, d.ly, 1e-3, 1.0, 6)
        assert int(s.item()) == b.PST_OK
        assert rel_err(to_host(t), ref) < TOL[1], p.shape


def test_sine_gordon_and_navier_stokes_stay_power_of_two():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    plan = b.Plan(96, 96, b.PST_R2C, b.PST_FP64, 1)
    u = torch.zeros(1, 96, 96, dtype=torch.float64, device="cuda")
    with pytest.raises(b.PstError, match="UNSUPPORTED"):
        plan.sg_step(u, u.clone(), inputs.PAPER_DOMAIN, 0.01, 1)
    with pytest.raises(b.PstError, match="UNSUPPORTED"):
        plan.ns_step(u, inputs.NS_DOMAIN, 1e-3, 1e-3, 1)
    with pytest.raises(b.PstError, match="UNSUPPORTED"):
        b.solve_batch([{"eq": "ns", "f0": u[0], "params": b.make_params("ns", inputs.NS_DOMAIN, 1e-3),
                        "nsteps": 1}])
    with pytest.raises(b.PstError, match="UNSUPPORTED"):
        b.Plan(4800 + 200, 16, b.PST_C2C, b.PST_FP64, 1)      # 5000: beyond the FP64 mixed-radix limit
