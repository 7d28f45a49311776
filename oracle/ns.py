"""Oracle: Crank-Nicolson with fixed-point iteration for 2D Navier-Stokes in
vorticity / stream-function form.

Equations (Section "The 2D Navier-Stokes Equation"), with the viscosity made
a parameter nu (the paper writes nu = 1):

    omega_t + psi_y omega_x - psi_x omega_y = nu Delta omega,
    Delta psi = -omega.

Scheme (Section "A Numerical Method for the 2D Navier-Stokes Equation"):
per time step the iterate omega^{n+1,k+1} solves, per Fourier mode,

    (w' - omega^n)/dt + nu |k|^2 (w' + omega^n)/2
        + (J(omega^{n+1,k}) + J(omega^n))/2 = 0,

J = psi_y omega_x - psi_x omega_y, starting from omega^{n+1,0} = omega^n and
stopping once integral (omega^{n+1,k} - omega^{n+1,k+1})^2 dxdy < tol.

Readings of the paper taken here:
  * nu is a parameter; the Table 4 error of 1.65e-5 is reproduced with
    nu = 0.1 (and not with the printed nu = 1);
  * the Jacobian is dealiased by the square 2/3 rule: its spectrum is set to
    zero where |m_x| or |m_y| > floor((n-1)/3) (not in the paper);
  * psi_hat = omega_hat/|k|^2 with psi_hat(0) = 0; first derivatives zero
    the Nyquist wavenumber;
  * J(omega^n) is evaluated once per step and reused in every iteration;
  * the iteration count is capped by max_iter (the paper gives no cap);
    fixed_iters > 0 runs exactly that many iterations regardless of tol.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


def _derivative_k(n, length):
    k = sp.wavenumbers(n, length)
    k[n // 2] = 0.0          # Nyquist wavenumber dropped for first derivatives
    return k


def _half_grids(shape, lx, ly):
    ny, nx = shape
    kx = sp.rwavenumbers(nx, lx)
    kx_d = kx.copy()
    kx_d[nx // 2] = 0.0
    ky = sp.wavenumbers(ny, ly)
    ky_d = _derivative_k(ny, ly)
    KX, KY = np.meshgrid(kx, ky, indexing="xy")
    KXd, KYd = np.meshgrid(kx_d, ky_d, indexing="xy")
    return KX * KX + KY * KY, KXd, KYd


def dealias_mask(shape):
    """1 where |m_x|, |m_y| <= floor((n-1)/3) on the [ny][nx/2+1] half grid."""
    ny, nx = shape
    mx = np.arange(nx // 2 + 1)
    my = np.abs(np.fft.fftfreq(ny, 1.0 / ny))
    MX, MY = np.meshgrid(mx, my, indexing="xy")
    return ((MX <= (nx - 1) // 3) & (MY <= (ny - 1) // 3)).astype(np.float64)


def stream_function_hat(w_hat, k2):
    """Solve Delta psi = -omega: psi_hat = omega_hat/|k|^2, psi_hat(0) = 0."""
    safe = np.where(k2 == 0.0, 1.0, k2)
    return np.where(k2 == 0.0, 0.0, w_hat / safe)


def jacobian_hat(w_hat, shape, lx, ly):
    """Dealiased spectrum of J = psi_y omega_x - psi_x omega_y."""
    k2, KXd, KYd = _half_grids(shape, lx, ly)
    psi_hat = stream_function_hat(w_hat, k2)
    psi_x = sp.irfft2(1j * KXd * psi_hat, shape)
    psi_y = sp.irfft2(1j * KYd * psi_hat, shape)
    om_x = sp.irfft2(1j * KXd * w_hat, shape)
    om_y = sp.irfft2(1j * KYd * w_hat, shape)
    J = psi_y * om_x - psi_x * om_y
    return dealias_mask(shape) * sp.rfft2(J)


def step(omega, lx, ly, dt, nu, tol=1e-10, max_iter=50, fixed_iters=0):
    """One Crank-Nicolson step with fixed-point iteration.

    Returns (omega^{n+1}, iterations, converged).
    """
    shape = omega.shape
    k2, _, _ = _half_grids(shape, lx, ly)
    w_n = sp.rfft2(omega)
    J_n = jacobian_hat(w_n, shape, lx, ly)
    w_k, J_k = w_n, J_n
    iters = 0
    converged = False
    while True:
        w_next = (((1.0 / dt) - 0.5 * nu * k2) * w_n - 0.5 * (J_k + J_n)) \
            / ((1.0 / dt) + 0.5 * nu * k2)
        iters += 1
        diff = sp.irfft2(w_k, shape) - sp.irfft2(w_next, shape)
        res = sp.integral(diff * diff, lx, ly)
        w_k = w_next
        if fixed_iters > 0:
            if iters == fixed_iters:
                converged = True
                break
        elif res < tol:
            converged = True
            break
        elif iters >= max_iter:
            break
        J_k = jacobian_hat(w_k, shape, lx, ly)
    return sp.irfft2(w_k, shape), iters, converged


def run(omega0, lx, ly, dt, nu, nsteps, tol=1e-10, max_iter=50, fixed_iters=0):
    """Advance omega0 by nsteps; returns (omega, iterations per step, all
    steps converged)."""
    omega = np.array(omega0, dtype=np.float64, copy=True)
    its = []
    ok = True
    for _ in range(nsteps):
        omega, it, conv = step(omega, lx, ly, dt, nu, tol, max_iter, fixed_iters)
        its.append(it)
        ok = ok and conv
    return omega, its, ok


def energy(omega, lx, ly):
    """Kinetic energy (1/2) integral |u|^2, u = (psi_y, -psi_x):
    |u_hat|^2 = |omega_hat|^2/|k|^2 by Parseval, mean mode excluded."""
    ny, nx = omega.shape
    KX, KY = sp.k_grids(nx, ny, lx, ly)
    k2 = KX * KX + KY * KY
    wh = sp.fft2(omega)
    safe = np.where(k2 == 0.0, 1.0, k2)
    s = np.sum(np.where(k2 == 0.0, 0.0, np.abs(wh) ** 2 / safe))
    return float(0.5 * lx * ly / float(nx * ny) ** 2 * s)


def enstrophy(omega, lx, ly):
    """(1/2) integral omega^2 dx dy."""
    return 0.5 * sp.integral(omega * omega, lx, ly)
