"""Pins for the oracle's spectral building blocks against brute force and
closed forms (no GPU)."""
import math

import numpy as np
import pytest

from oracle import spectral as sp


def naive_dft2(f, sign=-1):
    """Direct O(nx^2 ny^2) sum: F[q,p] = sum_{y,x} f[y,x] exp(sign*2*pi*i*(p*x/nx + q*y/ny))."""
    ny, nx = f.shape
    x = np.arange(nx)
    y = np.arange(ny)
    ex = np.exp(sign * 2j * math.pi * np.outer(x, x) / nx)   # [p][x]
    ey = np.exp(sign * 2j * math.pi * np.outer(y, y) / ny)   # [q][y]
    out = np.zeros((ny, nx), dtype=np.complex128)
    for q in range(ny):
        for p in range(nx):
            out[q, p] = np.sum(f * ey[q][:, None] * ex[p][None, :])
    return out


@pytest.mark.parametrize("nx,ny", [(4, 4), (8, 8), (16, 16), (8, 4), (4, 16), (6, 10), (15, 12), (5, 9), (20, 6)])
def test_fft2_matches_naive_dft(nx, ny):
    rng = np.random.default_rng(nx * 100 + ny)
    f = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    F = naive_dft2(f, -1)
    assert np.max(np.abs(sp.fft2(f) - F)) < 1e-12 * np.max(np.abs(F))
    # inverse: unnormalised +i sum divided by nx*ny
    G = naive_dft2(F, +1) / (nx * ny)
    assert np.max(np.abs(sp.ifft2(F) - G)) < 1e-13
    assert np.max(np.abs(sp.ifft2(F) - f)) < 1e-13


@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 4)])
def test_rfft2_is_half_of_full(nx, ny):
    rng = np.random.default_rng(7)
    f = rng.standard_normal((ny, nx))
    F = naive_dft2(f.astype(np.complex128), -1)
    assert np.max(np.abs(sp.rfft2(f) - F[:, : nx // 2 + 1])) < 1e-12
    assert np.max(np.abs(sp.irfft2(sp.rfft2(f), f.shape) - f)) < 1e-13


def test_wavenumbers_order_and_nyquist():
    k = sp.wavenumbers(8, 2 * math.pi)
    assert list(k) == [0, 1, 2, 3, -4, -3, -2, -1]
    kr = sp.rwavenumbers(8, 4 * math.pi)
    assert np.allclose(kr, [0, 0.5, 1.0, 1.5, 2.0])


def test_derivative_of_single_mode():
    # d/dx exp(i*3*x) on [0, 2pi) equals 3i*exp(i*3x); k*f_hat picks it up exactly
    n, L = 16, 2 * math.pi
    x = np.arange(n) * L / n
    f = np.exp(3j * x)[None, :] * np.ones((n, 1))
    KX, KY = sp.k_grids(n, n, L, L)
    df = sp.ifft2(1j * KX * sp.fft2(f))
    assert np.max(np.abs(df - 3j * f)) < 1e-13


def test_quadrature_and_parseval_closed_forms():
    # integral of exp(-2 r^2) over a resolved periodic box = pi/2;
    # integral |grad exp(-r^2)|^2 = pi.
    n, L = 128, 16.0
    x = -L / 2 + np.arange(n) * L / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    g = np.exp(-(X * X + Y * Y))
    assert abs(sp.integral(g * g, L, L) - math.pi / 2) < 1e-12
    assert abs(sp.grad_sq_integral(sp.fft2(g), L, L) - math.pi) < 1e-10


@pytest.mark.parametrize("n", [5, 6, 9, 12, 15])
def test_wavenumbers_of_lengths_that_are_not_powers_of_two(n):
    # fftfreq order for any n: 0..ceil(n/2)-1, then the negative ones; an
    # even n keeps -n/2 (the Nyquist mode), an odd n has none
    m = [round(k / (2 * math.pi)) for k in sp.wavenumbers(n, 1.0)]
    assert m == [j if j < (n + 1) // 2 else j - n for j in range(n)]
    assert list(np.round(sp.rwavenumbers(n, 1.0) / (2 * math.pi))) == list(range(n // 2 + 1))
