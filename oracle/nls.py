"""Oracle: split-step Fourier method for the 2D cubic NLS.

Equation (eq. nls, Section "The Cubic Nonlinear Schrodinger Equation"),
with the nonlinearity coefficient made a parameter g:

    i psi_t + psi_xx + psi_yy = g |psi|^2 psi,     g = +1 as eq. nls prints it.

Scheme (Section "A Numerical Method for the Nonlinear Schrodinger
Equation"): a linear half step solved exactly in Fourier space, a full
nonlinear step solved exactly in physical space, another linear half step.

Readings of the paper taken here:
  * the half-step multiplier is exp(-i |k|^2 dt/2); the paper's formula
    drops the 1/2 although its text says "half a time step";
  * the nonlinear sub-step of i psi_t = g|psi|^2 psi is
    psi <- exp(-i g |psi|^2 dt) psi, with |psi|^2 of the field entering the
    sub-step (it is invariant during it); the paper prints exp(+i...), which
    is the g = -1 (focusing) case;
  * the energy conserved by the g-equation is
    E = integral |grad psi|^2/2 + g |psi|^4/4; g = -1 gives the paper's
    eq. nlsmassenergy.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


def linear_substep(psi, lx, ly, tau):
    """Exact solution of eq. linSch, i psi_t + Delta psi = 0, over time tau:
    psi_hat <- exp(-i (kx^2+ky^2) tau) psi_hat."""
    ny, nx = psi.shape
    KX, KY = sp.k_grids(nx, ny, lx, ly)
    return sp.ifft2(np.exp(-1j * (KX * KX + KY * KY) * tau) * sp.fft2(psi))


def nonlinear_substep(psi, g, tau):
    """Exact solution of i psi_t = g |psi|^2 psi over time tau."""
    return np.exp(-1j * g * np.abs(psi) ** 2 * tau) * psi


def step(psi, lx, ly, dt, g):
    """One Strang step: L(dt/2) N(dt) L(dt/2)."""
    psi = linear_substep(psi, lx, ly, 0.5 * dt)
    psi = nonlinear_substep(psi, g, dt)
    return linear_substep(psi, lx, ly, 0.5 * dt)


def mass(psi, lx, ly):
    """integral |psi|^2 dx dy (eq. nlsmassenergy, first quantity)."""
    return sp.integral(np.abs(psi) ** 2, lx, ly)


def energy(psi, lx, ly, g):
    """integral |grad psi|^2/2 + g |psi|^4/4 dx dy (eq. nlsmassenergy with
    the g reading); the gradient term by Parseval."""
    kinetic = 0.5 * sp.grad_sq_integral(sp.fft2(psi), lx, ly)
    potential = 0.25 * g * sp.integral(np.abs(psi) ** 4, lx, ly)
    return kinetic + potential


def run(psi0, lx, ly, dt, g, nsteps, diag_every=0):
    """Advance psi0 by nsteps Strang steps.

    Returns (psi, diags) where diags is a list of (step, mass, energy) taken
    at step 0 and every diag_every steps (empty if diag_every == 0).
    """
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    diags = []
    if diag_every:
        diags.append((0, mass(psi, lx, ly), energy(psi, lx, ly, g)))
    for n in range(1, nsteps + 1):
        psi = step(psi, lx, ly, dt, g)
        if diag_every and n % diag_every == 0:
            diags.append((n, mass(psi, lx, ly), energy(psi, lx, ly, g)))
    return psi, diags
