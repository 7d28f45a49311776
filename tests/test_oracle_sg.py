"""Pins for the sine-Gordon oracle (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import sg
from paper_1206_3215_amd import inputs


def test_uniform_field_is_the_pendulum_leapfrog():
    # A spatially uniform field has only the k = 0 mode, where the scheme is
    # the textbook leapfrog for the pendulum u'' = -sin u, with the Taylor
    # start u^1 = u^0 + dt v^0 - dt^2 sin(u^0)/2.
    n, L, dt = 16, 10 * math.pi, 0.05
    u0 = np.full((n, n), 1.1)
    v0 = np.full((n, n), -0.3)
    a = u0[0, 0]
    b = a + dt * v0[0, 0] - 0.5 * dt * dt * math.sin(a)
    u1 = sg.start(u0, v0, L, L, dt)
    assert np.max(np.abs(u1 - b)) < 1e-14
    um, uc = u0, u1
    for _ in range(300):
        a, b = b, 2 * b - a - dt * dt * math.sin(b)
    um, uc = sg.run(u0, u1, L, L, dt, 300)
    assert np.max(np.abs(uc - b)) < 1e-12 and np.max(np.abs(um - a)) < 1e-12


def _mode(n, L, mx, my, eps):
    X, Y = inputs.grid(n, n, inputs.Domain(L, L, 0.0, 0.0))
    kx, ky = 2 * math.pi * mx / L, 2 * math.pi * my / L
    return eps * np.cos(kx * X + ky * Y), kx * kx + ky * ky


def test_small_mode_follows_klein_gordon_to_second_order():
    # eps*cos(k.x) with eps tiny: sin u = u to 1e-21, so the exact solution of
    # eq. sg is eps*cos(k.x)*cos(sqrt(|k|^2+1) t).  The scheme must converge
    # to it at second order; the printed "+Delta" sign would make the mode
    # grow instead.
    n, L, eps, T = 16, 2 * math.pi, 1e-7, 2.0
    u0, k2 = _mode(n, L, 3, 2, eps)
    omega = math.sqrt(k2 + 1.0)
    errs = []
    for nsteps in (200, 400, 800):
        dt = T / nsteps
        u1 = sg.start(u0, np.zeros_like(u0), L, L, dt)
        _, uT = sg.run(u0, u1, L, L, dt, nsteps - 1)
        errs.append(np.max(np.abs(uT - u0 * math.cos(omega * T))) / eps)
    assert errs[-1] < 2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_linear_hamiltonian_conserved_to_rounding():
    # With the sine term removed the scheme is the (1,2,1)/4-weighted wave
    # scheme, whose staggered energy H^{n+1/2} is an exact invariant (only for
    # these weights), so it must hold to rounding.
    d = inputs.PAPER_DOMAIN
    u0, v0 = inputs.sg_gaussian(64, 64, d, seed=1, abs_noise=1e-2)
    dt = 0.05
    u1 = sg.start(u0, v0, d.lx, d.ly, dt, forcing=False)
    h0 = sg.hamiltonian(u0, u1, d.lx, d.ly, dt, forcing=False)[3]
    a, b = sg.run(u0, u1, d.lx, d.ly, dt, 60, forcing=False)
    h1 = sg.hamiltonian(a, b, d.lx, d.ly, dt, forcing=False)[3]
    assert abs(h1 / h0 - 1) < 1e-12


def test_initial_hamiltonian_closed_form():
    # u = A exp(-r^2), u_t = 0:  H = A^2 pi/2 + sum_j (-1)^(j+1) A^(2j) pi/((2j)! 2j)
    A = 0.5
    d = inputs.PAPER_DOMAIN
    u0, _ = inputs.sg_gaussian(256, 256, d, seed=None, amp=A)
    series = sum((-1) ** (j + 1) * A ** (2 * j) * math.pi / (math.factorial(2 * j) * 2 * j)
                 for j in range(1, 12))
    h = sg.hamiltonian(u0, u0, d.lx, d.ly, 0.01)
    assert abs(h[3] - (A * A * math.pi / 2 + series)) < 1e-12
    assert h[0] == 0.0


def test_hamiltonian_six_figures_and_second_order_drift(golden_dir):
    # Paper's bar (Table 3 workload: 500 steps of dt = 1e-3 on [-5pi,5pi)^2):
    # the final Hamiltonian within 6 significant figures.  The drift comes
    # from the explicit sine term and must scale as dt^2.
    bars = json.load(open(os.path.join(golden_dir, "paper_conservation.json")))["sg"]
    d = inputs.PAPER_DOMAIN
    u0, v0 = inputs.sg_gaussian(64, 64, d, seed=0)
    drift = {}
    for dt, steps in ((1e-3, 500), (2e-3, 250)):
        u1 = sg.start(u0, v0, d.lx, d.ly, dt)
        h0 = sg.hamiltonian(u0, u1, d.lx, d.ly, dt)[3]
        a, b = sg.run(u0, u1, d.lx, d.ly, dt, steps - 1)
        drift[dt] = sg.hamiltonian(a, b, d.lx, d.ly, dt)[3] / h0 - 1
    assert abs(drift[1e-3]) < 0.5 * 10.0 ** (1 - bars["hamiltonian_significant_figures"])
    assert 3.8 < drift[2e-3] / drift[1e-3] < 4.2, drift
