"""Fourier pseudospectral building blocks (Section "Fourier Pseudospectral
Methods"): derivatives become multiplication by i*k in Fourier space.

Conventions (not fixed by the paper; readings listed in the design notes):
  * forward transform unnormalised with kernel exp(-i k.x), inverse scaled by
    1/(nx*ny) -- scipy.fft's default;
  * wavenumbers k = 2*pi*m/L with m in {0..n/2-1, -n/2..-1} (numpy fftfreq
    order), so the Nyquist mode carries k^2 = (pi*n/L)^2;
  * quadrature of a periodic field is dx*dy*sum (spectrally accurate), and
    gradient integrals use Parseval:  integral |grad f|^2 =
    lx*ly/(nx*ny)^2 * sum |k|^2 |f_hat|^2.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

WORKERS = os.cpu_count() or 1


def fft2(f):
    return sfft.fft2(f, workers=WORKERS)


def ifft2(F):
    return sfft.ifft2(F, workers=WORKERS)


def rfft2(f):
    return sfft.rfft2(f, workers=WORKERS)


def irfft2(F, shape):
    return sfft.irfft2(F, s=shape, workers=WORKERS)


def wavenumbers(n: int, length: float) -> np.ndarray:
    """k_m = 2*pi*m/length, m in fftfreq order."""
    return 2.0 * math.pi * np.fft.fftfreq(n, 1.0 / n) / length


def rwavenumbers(n: int, length: float) -> np.ndarray:
    """k_m for the half axis of a real transform, m = 0..n/2."""
    return 2.0 * math.pi * np.arange(n // 2 + 1, dtype=np.float64) / length


def k_grids(nx: int, ny: int, lx: float, ly: float):
    """(KX, KY) on the full [ny][nx] spectral grid."""
    return np.meshgrid(wavenumbers(nx, lx), wavenumbers(ny, ly), indexing="xy")


def rk_grids(nx: int, ny: int, lx: float, ly: float):
    """(KX, KY) on the half [ny][nx/2+1] grid of a real transform along x."""
    return np.meshgrid(rwavenumbers(nx, lx), wavenumbers(ny, ly), indexing="xy")


def cell_area(shape, lx: float, ly: float) -> float:
    ny, nx = shape
    return (lx / nx) * (ly / ny)


def integral(f, lx: float, ly: float) -> float:
    """dx*dy*sum f over the periodic grid."""
    return float(cell_area(f.shape, lx, ly) * np.sum(f))


def grad_sq_integral(f_hat, lx: float, ly: float) -> float:
    """integral |grad f|^2 from the full 2D transform f_hat (Parseval)."""
    ny, nx = f_hat.shape
    KX, KY = k_grids(nx, ny, lx, ly)
    return float(lx * ly / float(nx * ny) ** 2
                 * np.sum((KX * KX + KY * KY) * np.abs(f_hat) ** 2))
