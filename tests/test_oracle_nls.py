"""Pins for the NLS split-step oracle (no GPU).

Closed forms and invariants fixed by the mathematics and the paper's
Results section; see oracle/nls.py for the readings they pin."""
import json
import math
import os

import numpy as np
import pytest

from oracle import nls
from paper_1206_3215_amd import inputs


def plane_wave(nx, ny, lx, ly, mx, my, A, g, t):
    x = np.arange(nx) * lx / nx
    y = np.arange(ny) * ly / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    kx, ky = 2 * math.pi * mx / lx, 2 * math.pi * my / ly
    return A * np.exp(1j * (kx * X + ky * Y - (kx * kx + ky * ky + g * abs(A) ** 2) * t))


@pytest.mark.parametrize("g", [1.0, -1.0, 0.0])
def test_plane_wave_exact_any_dt(g):
    # Each sub-step is exact on a plane wave, so Strang splitting reproduces
    # psi = A exp(i(k.x - (|k|^2 + g|A|^2) t)) to rounding for any dt.
    # Non-square grid and box so that a swapped kx/ky is caught.
    nx, ny, lx, ly = 32, 16, 6.0, 4.0
    A, mx, my, dt, n = 0.7 + 0.2j, 3, -2, 0.01, 200
    psi0 = plane_wave(nx, ny, lx, ly, mx, my, A, g, 0.0)
    psi, _ = nls.run(psi0, lx, ly, dt, g, n)
    exact = plane_wave(nx, ny, lx, ly, mx, my, A, g, n * dt)
    assert np.max(np.abs(psi - exact)) < 1e-11


def test_linear_superposition_closed_form():
    # g = 0: each Fourier mode rotates by exp(-i |k|^2 t), independently.
    nx, ny, lx, ly = 16, 32, 5.0, 7.0
    t = 0.37
    a = plane_wave(nx, ny, lx, ly, 2, 5, 0.3, 0.0, 0.0) + plane_wave(nx, ny, lx, ly, -4, 1, 0.5j, 0.0, 0.0)
    e = plane_wave(nx, ny, lx, ly, 2, 5, 0.3, 0.0, t) + plane_wave(nx, ny, lx, ly, -4, 1, 0.5j, 0.0, t)
    psi, _ = nls.run(a, lx, ly, t / 10, 0.0, 10)
    assert np.max(np.abs(psi - e)) < 1e-12


def test_gaussian_initial_mass_and_energy_closed_form():
    # psi = 0.5 exp(-r^2): mass = pi/8, energy = pi/8 + g*pi/256 (resolved grid).
    d = inputs.NLS_SMALL_DOMAIN
    psi = inputs.nls_gaussian(256, 256, d, seed=None)
    for g in (1.0, -1.0):
        assert abs(nls.mass(psi, d.lx, d.ly) - math.pi / 8) < 1e-12
        assert abs(nls.energy(psi, d.lx, d.ly, g) - (math.pi / 8 + g * math.pi / 256)) < 1e-12


def test_mass_conserved_and_energy_six_figures(golden_dir):
    # Small workload: 64^2 on [-8pi,8pi)^2, seeded noise, dt 0.0025, 200 steps,
    # diagnostics every 20 steps.  Bars from the paper's Results section.
    bars = json.load(open(os.path.join(golden_dir, "paper_conservation.json")))["nls"]
    d = inputs.NLS_SMALL_DOMAIN
    psi0 = inputs.nls_gaussian(64, 64, d, seed=0)
    _, diags = nls.run(psi0, d.lx, d.ly, 0.0025, 1.0, 200, diag_every=20)
    m = np.array([x[1] for x in diags])
    e = np.array([x[2] for x in diags])
    assert len(diags) == 11
    assert np.max(np.abs(m / m[0] - 1)) < bars["mass_rel_drift_max"]
    assert np.max(np.abs(e / e[0] - 1)) < 0.5 * 10.0 ** (1 - bars["energy_significant_figures"])


def test_time_reversible():
    d = inputs.PAPER_DOMAIN
    psi0 = inputs.nls_gaussian(64, 64, d, seed=3)
    fwd, _ = nls.run(psi0, d.lx, d.ly, 1e-3, 1.0, 40)
    back, _ = nls.run(fwd, d.lx, d.ly, -1e-3, 1.0, 40)
    assert np.max(np.abs(back - psi0)) < 1e-12


def test_second_order_in_time():
    # Error against a fine-step reference drops by ~4 per halving of dt.
    d = inputs.Domain.centered_square(8.0)
    psi0 = 1.5 * inputs.nls_gaussian(32, 32, d, seed=None)
    T = 0.2
    ref, _ = nls.run(psi0, d.lx, d.ly, T / 256, 1.0, 256)
    errs = []
    for n in (8, 16, 32):
        psi, _ = nls.run(psi0, d.lx, d.ly, T / n, 1.0, n)
        errs.append(np.max(np.abs(psi - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


@pytest.mark.parametrize("nx,ny", [(12, 20), (15, 9)])
def test_plane_wave_exact_on_grids_that_are_not_powers_of_two(nx, ny):
    # the scheme and the pin are the same on any grid: 2^a 3^b 5^c lengths,
    # odd ones included, where the positive-frequency range differs
    lx, ly, A, mx, my, dt, n = 5.0, 3.0, 0.6 - 0.3j, -4, 3, 0.02, 60
    psi0 = plane_wave(nx, ny, lx, ly, mx, my, A, 1.0, 0.0)
    got, _ = nls.run(psi0, lx, ly, dt, 1.0, n)
    exact = plane_wave(nx, ny, lx, ly, mx, my, A, 1.0, dt * n)
    assert np.max(np.abs(got - exact)) < 1e-12
