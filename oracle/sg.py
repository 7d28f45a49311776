"""Oracle: three-level scheme for the 2D sine-Gordon equation.

Equation (eq. sg):  u_tt - Delta u = -sin u.

Scheme (eq. sgmethodunformatted, Section "A Numerical Method for the
Sine-Gordon Equation"): central difference in time, the Laplacian acting on
the (1,2,1)/4 average of the three time levels, explicit -sin u^n.

Readings of the paper taken here:
  * sign of the Laplacian term.  The printed scheme carries "+Delta(...)",
    which discretises u_tt + Delta u = -sin u and contradicts eq. sg; it is
    also unconditionally unstable for the stiff modes.  The scheme below uses
    -Delta, i.e. +|k|^2 in Fourier space, matching eq. sg.  The structure
    (central difference, (1,2,1)/4 weights, explicit sine) is the paper's.
  * start-up.  The paper does not say how the second level is formed from
    (u^0, u_t^0).  Here the centred velocity u^{-1} = u^1 - 2 dt v^0 is
    substituted into the scheme at n = 0 and the result is solved for u^1.
  * the discrete Hamiltonian is the staggered H^{n+1/2} of hamiltonian().
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


def _k2(shape, lx, ly):
    ny, nx = shape
    KX, KY = sp.rk_grids(nx, ny, lx, ly)
    return KX * KX + KY * KY


def start(u0, v0, lx, ly, dt, forcing=True):
    """Second time level u^1 from u^0 and u_t(0) = v0.

    Per Fourier mode, with u^{-1} = u^1 - 2 dt v^0 substituted into
        (u^1 - 2u^0 + u^{-1})/dt^2 + |k|^2 (u^1 + 2u^0 + u^{-1})/4 = -s^0,
    i.e.  u^1 (2/dt^2 + |k|^2/2)
            = 2u^0/dt^2 + 2 v^0/dt - |k|^2 (2u^0 - 2 dt v^0)/4 - s^0.
    """
    shape = u0.shape
    k2 = _k2(shape, lx, ly)
    u0h = sp.rfft2(u0)
    v0h = sp.rfft2(v0)
    s0h = sp.rfft2(np.sin(u0)) if forcing else np.zeros_like(u0h)
    rhs = 2.0 * u0h / dt ** 2 + 2.0 * v0h / dt - k2 * (2.0 * u0h - 2.0 * dt * v0h) / 4.0 - s0h
    u1h = rhs / (2.0 / dt ** 2 + k2 / 2.0)
    return sp.irfft2(u1h, shape)


def step(u_prev, u_curr, lx, ly, dt, forcing=True):
    """u^{n+1} from (u^{n-1}, u^n), solving per Fourier mode
        (u^{n+1} - 2u^n + u^{n-1})/dt^2 + |k|^2 (u^{n+1} + 2u^n + u^{n-1})/4
            = -FFT(sin u^n).
    """
    shape = u_curr.shape
    k2 = _k2(shape, lx, ly)
    unh = sp.rfft2(u_curr)
    umh = sp.rfft2(u_prev)
    snh = sp.rfft2(np.sin(u_curr)) if forcing else np.zeros_like(unh)
    lhs = 1.0 / dt ** 2 + k2 / 4.0
    rhs = (2.0 / dt ** 2 - k2 / 2.0) * unh - (1.0 / dt ** 2 + k2 / 4.0) * umh - snh
    return sp.irfft2(rhs / lhs, shape)


def run(u_prev, u_curr, lx, ly, dt, nsteps, forcing=True):
    """Advance the pair (u^{n-1}, u^n) by nsteps; returns the new pair."""
    a = np.array(u_prev, dtype=np.float64, copy=True)
    b = np.array(u_curr, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        a, b = b, step(a, b, lx, ly, dt, forcing)
    return a, b


def hamiltonian(u_n, u_np1, lx, ly, dt, forcing=True):
    """Staggered discrete Hamiltonian H^{n+1/2} of H = integral
    (u_t^2 + |grad u|^2)/2 + (1 - cos u), with u_t = (u^{n+1}-u^n)/dt,
    grad of the mean ubar = (u^{n+1}+u^n)/2 (Parseval), and the potential
    averaged over the two levels.

    Returns (kinetic, gradient, potential, total); potential is 0 when
    forcing is False (the linear wave equation).
    """
    kinetic = 0.5 * sp.integral(((u_np1 - u_n) / dt) ** 2, lx, ly)
    gradient = 0.5 * sp.grad_sq_integral(sp.fft2(0.5 * (u_np1 + u_n)), lx, ly)
    if forcing:
        potential = sp.integral(0.5 * (1.0 - np.cos(u_np1)) + 0.5 * (1.0 - np.cos(u_n)), lx, ly)
    else:
        potential = 0.0
    return kinetic, gradient, potential, kinetic + gradient + potential
