"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle.

This module builds initial conditions and request mixes only; it holds none
of the time-stepping schemes' arithmetic and imports neither the oracle nor
the HIP binding.  Every array is float64/complex128, laid out row-major as
``[ny][nx]`` (x is the fast axis); FP32 runs round these once.

Grid convention (periodic, right end point excluded): ``x_j = x0 + j*lx/nx``.

Workload shapes follow the paper's benchmark problems (Section "An Overview
of The Equations" and Tables 2-4): a Gaussian NLS pulse on [-5pi,5pi)^2, a
Gaussian sine-Gordon bump on the same square, and 2D Navier-Stokes on
[0,1)^2 with either the Taylor-Green vortex (eq. TaylorGreen) or a
random-phase vorticity field.  The paper prints no noise or random-phase
recipe; the ones below are this project's synthetic stand-ins.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Domain:
    """Periodic rectangle: x in [x0, x0+lx), y in [y0, y0+ly)."""

    lx: float
    ly: float
    x0: float
    y0: float

    @staticmethod
    def centered_square(length: float) -> "Domain":
        return Domain(length, length, -0.5 * length, -0.5 * length)

    @staticmethod
    def unit_square() -> "Domain":
        return Domain(1.0, 1.0, 0.0, 0.0)


# Domains of the paper's timing tables and of the larger synthetic workloads.
NLS_SMALL_DOMAIN = Domain.centered_square(16.0 * math.pi)   # [-8pi, 8pi)^2
PAPER_DOMAIN = Domain.centered_square(10.0 * math.pi)       # [-5pi, 5pi)^2
NS_DOMAIN = Domain.unit_square()                            # [0, 1)^2


def grid(nx: int, ny: int, d: Domain):
    """Return (X, Y) of shape [ny][nx] with x_j = x0 + j*lx/nx."""
    x = d.x0 + np.arange(nx, dtype=np.float64) * (d.lx / nx)
    y = d.y0 + np.arange(ny, dtype=np.float64) * (d.ly / ny)
    return np.meshgrid(x, y, indexing="xy")


def noise(nx: int, ny: int, seed: int) -> np.ndarray:
    """Standard normal field xi[ny][nx] from numpy's PCG64 generator."""
    return np.random.default_rng(seed).standard_normal((ny, nx))


def nls_gaussian(nx: int, ny: int, d: Domain, seed: int | None,
                 amp: float = 0.5, rel_noise: float = 0.01) -> np.ndarray:
    """psi0 = amp*exp(-(x^2+y^2))*(1 + rel_noise*xi), complex128."""
    X, Y = grid(nx, ny, d)
    env = amp * np.exp(-(X * X + Y * Y))
    if seed is None or rel_noise == 0.0:
        return env.astype(np.complex128)
    return (env * (1.0 + rel_noise * noise(nx, ny, seed))).astype(np.complex128)


def sg_gaussian(nx: int, ny: int, d: Domain, seed: int | None,
                amp: float = 0.5, abs_noise: float = 1e-3):
    """(u0, v0): u0 = amp*exp(-(x^2+y^2)) + abs_noise*xi, v0 = 0 (float64)."""
    X, Y = grid(nx, ny, d)
    u0 = amp * np.exp(-(X * X + Y * Y))
    if seed is not None and abs_noise != 0.0:
        u0 = u0 + abs_noise * noise(nx, ny, seed)
    return u0, np.zeros_like(u0)


def taylor_green(n: int, t: float = 0.0, nu: float = 1.0) -> np.ndarray:
    """Vorticity of the Taylor-Green vortex on [0,1)^2 (eq. TaylorGreen).

    The paper writes the unit-viscosity decay exp(-8 pi^2 t); with viscosity
    nu the factor is exp(-8 pi^2 nu t).
    """
    X, Y = grid(n, n, NS_DOMAIN)
    return (4.0 * math.pi * np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y)
            * math.exp(-8.0 * math.pi ** 2 * nu * t))


def dealias_cutoff(n: int) -> int:
    """Largest |m| kept by the square 2/3 truncation: floor((n-1)/3)."""
    return (n - 1) // 3


def ns_random_phase(n: int, seed: int, k_peak: float = 8.0) -> np.ndarray:
    """Random-phase vorticity on [0,1)^2 with unit kinetic energy.

    Integer wavenumbers m = (mx, my) in FFT order, shell kappa = |m|.  Each
    mode gets amplitude |k| * sqrt(E(kappa)/(pi*kappa)) with
    E(kappa) = kappa^4 exp(-(kappa/k_peak)^2), k = 2*pi*m, and a phase drawn
    uniformly from [0, 2pi).  Modes outside the square 2/3 truncation are
    dropped; the real part of the inverse transform is then rescaled so that
    (1/2) * integral |u|^2 = 1, with u the velocity of the stream function.
    """
    m = np.fft.fftfreq(n, 1.0 / n)
    MX, MY = np.meshgrid(m, m, indexing="xy")
    kappa = np.hypot(MX, MY)
    theta = np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, (n, n))
    with np.errstate(divide="ignore", invalid="ignore"):
        e = kappa ** 4 * np.exp(-(kappa / k_peak) ** 2)
        amp = 2.0 * math.pi * kappa * np.sqrt(e / (math.pi * kappa))
    amp[0, 0] = 0.0
    K = dealias_cutoff(n)
    amp[(np.abs(MX) > K) | (np.abs(MY) > K)] = 0.0
    w = np.real(np.fft.ifft2(amp * np.exp(1j * theta))) * (n * n)
    # Kinetic energy of w: (1/2) sum_{k != 0} |w_hat|^2 / |k|^2 / n^4 on [0,1)^2.
    w_hat = np.fft.fft2(w)
    k2 = (2.0 * math.pi) ** 2 * (MX * MX + MY * MY)
    k2[0, 0] = 1.0
    energy = 0.5 * np.sum(np.abs(w_hat) ** 2 / k2 * (kappa > 0)) / float(n) ** 4
    return w / math.sqrt(energy)


# ----------------------------------------------------------------------------
# Request mix for the continuous-batching loop.

@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    eq: str          # "nls" | "sg" | "ns"
    n: int           # grid is n x n
    steps: int
    arrival_s: float


def serving_mix(count: int = 512, rate_hz: float = 10.0, seed: int = 12345,
                log2n_range=(7, 11), steps_range=(100, 2000)) -> list[Request]:
    """Poisson arrivals at rate_hz; equation uniform over {nls, sg, ns};
    n = 2**e with e uniform on log2n_range (inclusive); steps uniform on
    steps_range (inclusive).  The initial-condition seed of request i is i."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    eqs = rng.integers(0, 3, count)
    es = rng.integers(log2n_range[0], log2n_range[1] + 1, count)
    steps = rng.integers(steps_range[0], steps_range[1] + 1, count)
    names = ("nls", "sg", "ns")
    return [Request(i, names[int(eqs[i])], 1 << int(es[i]), int(steps[i]),
                    float(arrivals[i])) for i in range(count)]
