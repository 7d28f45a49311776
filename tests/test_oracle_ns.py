"""Pins for the Navier-Stokes oracle (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ns
from oracle import spectral as sp
from paper_1206_3215_amd import inputs


@pytest.mark.parametrize("n", [64, 128])
def test_paper_table4_taylor_green_max_error(golden_dir, n):
    # Worked example printed with Table 4: 20 steps of dt = 1.25e-3 on [0,1]^2,
    # tol 1e-10, max error 1.65e-5 vs the exact Taylor-Green vortex on every
    # grid (reproduced with nu = 0.1, see the golden file's reading).
    g = json.load(open(os.path.join(golden_dir, "paper_table4_taylor_green.json")))
    nu = 0.1
    w0 = inputs.taylor_green(n, 0.0, nu)
    w, its, ok = ns.run(w0, 1.0, 1.0, g["dt"], nu, g["steps"], tol=g["tol"])
    assert ok
    exact = inputs.taylor_green(n, g["steps"] * g["dt"], nu)
    err = np.max(np.abs(w - exact))
    assert abs(err - g["max_error"]) < 0.5 * 10.0 ** (-g["printed_digits"] + 1) * 1e-5


def test_taylor_green_crank_nicolson_ratio_per_step():
    # J vanishes on the Taylor-Green vortex, so each step multiplies it by
    # the Crank-Nicolson factor (1 - dt nu |k|^2/2)/(1 + dt nu |k|^2/2), |k|^2 = 8 pi^2.
    n, dt, nu = 32, 1e-3, 1e-3 * 37
    w0 = inputs.taylor_green(n)
    w1, its, ok = ns.step(w0, 1.0, 1.0, dt, nu)
    k2 = 8 * math.pi ** 2
    rho = (1 - 0.5 * dt * nu * k2) / (1 + 0.5 * dt * nu * k2)
    assert ok and its <= 2
    assert np.max(np.abs(w1 - rho * w0)) < 1e-13


def test_taylor_green_initial_energy_enstrophy():
    w = inputs.taylor_green(64)
    assert abs(ns.energy(w, 1.0, 1.0) - 0.25) < 1e-13
    assert abs(ns.enstrophy(w, 1.0, 1.0) - 2 * math.pi ** 2) < 1e-11


def test_poisson_single_mode():
    # Delta psi = -omega for omega = cos(2 pi (3x + 2y)):  psi = omega/(4 pi^2 13)
    n = 32
    X, Y = inputs.grid(n, n, inputs.NS_DOMAIN)
    w = np.cos(2 * math.pi * (3 * X + 2 * Y))
    k2, _, _ = ns._half_grids(w.shape, 1.0, 1.0)
    psi = sp.irfft2(ns.stream_function_hat(sp.rfft2(w), k2), w.shape)
    assert np.max(np.abs(psi - w / (4 * math.pi ** 2 * 13))) < 1e-15


def test_jacobian_closed_form_non_square():
    # psi = A sin(p x) + B cos(q y), omega = -Delta psi:
    # J = psi_y omega_x - psi_x omega_y = A B p q (q^2 - p^2) cos(p x) sin(q y).
    nx, ny, lx, ly = 32, 16, 2.0, 1.0
    p, q = 2 * math.pi * 3 / lx, 2 * math.pi * 2 / ly
    A, B = 0.7, -1.3
    X, Y = inputs.grid(nx, ny, inputs.Domain(lx, ly, 0.0, 0.0))
    w = A * p * p * np.sin(p * X) + B * q * q * np.cos(q * Y)
    J = sp.irfft2(ns.jacobian_hat(sp.rfft2(w), w.shape, lx, ly), w.shape)
    exact = A * B * p * q * (q * q - p * p) * np.cos(p * X) * np.sin(q * Y)
    assert np.max(np.abs(J - exact)) < 1e-10 * np.max(np.abs(exact))


def test_dealiased_jacobian_invariants():
    # For band-limited fields the 2/3-truncated Jacobian is orthogonal to
    # omega and to psi (discrete form of integral omega J = integral psi J = 0).
    n = 64
    w = inputs.ns_random_phase(n, seed=5)
    wh = sp.rfft2(w)
    J = sp.irfft2(ns.jacobian_hat(wh, w.shape, 1.0, 1.0), w.shape)
    k2, _, _ = ns._half_grids(w.shape, 1.0, 1.0)
    psi = sp.irfft2(ns.stream_function_hat(wh, k2), w.shape)
    scale = np.sqrt(np.sum(J * J))
    assert abs(np.sum(w * J)) < 1e-12 * scale * np.sqrt(np.sum(w * w))
    assert abs(np.sum(psi * J)) < 1e-12 * scale * np.sqrt(np.sum(psi * psi))


def test_fixed_point_solves_crank_nicolson_within_tol():
    # At convergence the accepted iterate satisfies the CN equation up to the
    # size of the last correction.
    n, dt, nu, tol = 64, 1e-3, 1e-3, 1e-12
    w0 = inputs.ns_random_phase(n, seed=2)
    w1, its, ok = ns.step(w0, 1.0, 1.0, dt, nu, tol=tol, max_iter=50)
    assert ok and its >= 2
    k2, _, _ = ns._half_grids(w0.shape, 1.0, 1.0)
    a, b = sp.rfft2(w0), sp.rfft2(w1)
    resid = (b - a) / dt + 0.5 * nu * k2 * (a + b) + 0.5 * (
        ns.jacobian_hat(a, w0.shape, 1.0, 1.0) + ns.jacobian_hat(b, w0.shape, 1.0, 1.0))
    r = sp.irfft2(resid, w0.shape)
    # |dt * residual| is of the size of the last fixed-point update (< sqrt(tol))
    assert np.sqrt(sp.integral((dt * r) ** 2, 1.0, 1.0)) < 10 * math.sqrt(tol)


def test_fixed_iters_and_not_converged_flag():
    w0 = inputs.ns_random_phase(32, seed=1)
    _, its, ok = ns.run(w0, 1.0, 1.0, 1e-3, 1e-3, 3, fixed_iters=2)
    assert its == [2, 2, 2] and ok
    _, its, ok = ns.run(w0, 1.0, 1.0, 1e-3, 1e-3, 1, tol=0.0, max_iter=3)
    assert its == [3] and not ok


def test_random_phase_input_unit_energy_and_band_limited():
    w = inputs.ns_random_phase(128, seed=7)
    assert abs(ns.energy(w, 1.0, 1.0) - 1.0) < 1e-12
    wh = sp.rfft2(w)
    assert np.max(np.abs(wh * (1 - ns.dealias_mask(w.shape)))) < 1e-9 * np.max(np.abs(wh))
    assert np.array_equal(w, inputs.ns_random_phase(128, seed=7))


def test_two_thirds_rule_removes_aliasing():
    # The 2/3 rule exists so that the truncated pseudo-spectral Jacobian equals
    # the truncation of the exact Jacobian.  Build omega as a handful of modes
    # with |m| <= K = floor((n-1)/3), evaluate its exact Jacobian analytically
    # on a 2n grid (no aliasing there), truncate to |m_x|,|m_y| <= K and
    # compare with the oracle on the n grid.
    n = 32
    K = (n - 1) // 3
    rng = np.random.default_rng(11)
    modes = [(int(rng.integers(-K, K + 1)), int(rng.integers(-K, K + 1)),
              rng.standard_normal(), rng.uniform(0, 2 * math.pi)) for _ in range(8)]
    modes = [m for m in modes if (m[0], m[1]) != (0, 0)]

    def fields(N):
        X, Y = inputs.grid(N, N, inputs.NS_DOMAIN)
        out = {k: np.zeros((N, N)) for k in ("w", "wx", "wy", "px", "py")}
        for mx, my, a, ph in modes:
            kx, ky = 2 * math.pi * mx, 2 * math.pi * my
            k2 = kx * kx + ky * ky
            arg = kx * X + ky * Y + ph
            out["w"] += a * np.cos(arg)
            out["wx"] += -a * kx * np.sin(arg)
            out["wy"] += -a * ky * np.sin(arg)
            out["px"] += -a / k2 * kx * np.sin(arg)
            out["py"] += -a / k2 * ky * np.sin(arg)
        return out

    f2 = fields(2 * n)
    J2 = f2["py"] * f2["wx"] - f2["px"] * f2["wy"]
    J2h = np.fft.rfft2(J2) / 4.0                    # spectrum scaled to an n-grid transform
    m2y = np.fft.fftfreq(2 * n, 1.0 / (2 * n)).astype(int)
    expect = np.zeros((n, n // 2 + 1), dtype=np.complex128)
    for iy, my in enumerate(np.fft.fftfreq(n, 1.0 / n).astype(int)):
        if abs(my) > K:
            continue
        jy = int(np.where(m2y == my)[0][0])
        expect[iy, : K + 1] = J2h[jy, : K + 1]
    w = fields(n)["w"]
    got = ns.jacobian_hat(sp.rfft2(w), w.shape, 1.0, 1.0)
    assert np.max(np.abs(got - expect)) < 1e-9 * np.max(np.abs(expect))


def test_fixed_point_diverges_at_stated_dt_and_contracts_at_quarter_dt():
    # Random-phase vorticity (unit energy, spectrum k^4 exp(-(k/8)^2)), nu 1e-3
    # on a 512^2 grid: with dt 1e-3 the fixed-point map's gain on the modes
    # near k* = sqrt(2/(dt nu)) is about dt |u| k*/2 ~ 1, the iteration stops
    # converging within two steps and the field blows up; with dt 2.5e-4 it
    # converges every step in a handful of iterations.
    w0 = inputs.ns_random_phase(512, seed=1)
    w, conv_flags = w0, []
    with np.errstate(all="ignore"):
        for _ in range(6):
            w, it, conv = ns.step(w, 1.0, 1.0, 1e-3, 1e-3, tol=1e-10, max_iter=30)
            conv_flags.append(conv)
    assert not all(conv_flags)
    assert not np.all(np.isfinite(w)) or np.max(np.abs(w)) > 10 * np.max(np.abs(w0))
    w = w0
    for _ in range(3):
        w, it, conv = ns.step(w, 1.0, 1.0, 2.5e-4, 1e-3, tol=1e-10, max_iter=30)
        assert conv and it <= 8
    assert np.all(np.isfinite(w))


def test_twin_experiment_record_bounds_the_parity_horizon(golden_dir):
    # The stored twin experiment (tests/golden/gen_refs.py twin: the oracle
    # against itself from a field perturbed by 1e-14 and 1e-7 of its maximum,
    # random-phase 1024^2, nu 1e-3, dt 2.5e-4) shows the predictability
    # horizon lies beyond the 240 steps at which the GPU parity tests compare:
    # both perturbations grow by less than 10x over those steps.
    import json
    rec = json.load(open(os.path.join(golden_dir, "ns_twin_1024.json")))
    r14, r7 = rec["rel_diff"]["p1e-14"], rec["rel_diff"]["p1e-7"]
    assert len(r14) == rec["steps"] >= 240
    assert max(r14[:240]) < 1e-13 and max(r7[:240]) < 1e-6
    assert all(2 <= it <= 12 for it in rec["iterations_ref"])
