"""Momentum predictor of the projection method (oracle; test infrastructure).

The paper solves the momentum equation by Chorin's projection (Sec. 4): first
a provisional velocity u^{n+1} from the momentum equation without the pressure
(eq. nopressmomentum), with u = 0 on the bottom wall and u = u_0 on the top
wall, then the pressure Poisson equation and the velocity correction (eqs.
pressuresolve and velocityupdate, oracle.step).  This module is the first
half:

    (u* - v^n)/dt = -(v^n . grad) v^n + nu * Lap v,          nu = 1/(rho Re_a),

with the viscous term theta-implicit (theta = 1/2 is the Crank-Nicolson
scheme the paper names for second order in time, theta = 1 backward Euler):

    (I - theta*dt*nu*L_D) u* = v^n - dt*(v^n . grad_h) v^n + (1-theta)*dt*nu*L_D v^n

for each component, on the interior rows j = 1..N-1; the wall rows j = 0, N
carry the Dirichlet data (x-component 0 at the bottom and U at the top,
y-component 0 on both: no penetration).  L_D is the 5-point Laplacian that
reads the wall rows as boundary values (no reflection); the advective
derivatives are central differences (Sec. 4).  The elastic and
phase-separation stresses of R (Sec. 4) are not part of this reduced
predictor.

The implicit operator as a matrix over all (N+1) x N nodes is identity on the
wall rows and 1 + 4s on the diagonal, -s on the four neighbours of an
interior node, s = theta*dt*nu/h^2; a wall value enters the first and last
interior rows as known data.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

from . import ops


def lap_dirichlet(x: np.ndarray) -> np.ndarray:
    """5-point Laplacian on the interior rows 1..N-1 with the wall rows of x as
    Dirichlet values (row values of Sec. 4.1: 4 at the centre, -1 at the four
    neighbours, times -1/h^2); zero on the wall rows."""
    n = ops.n_of(x)
    h = x.dtype.type(1) / n
    y = np.zeros_like(x)
    c = x[1:-1]
    y[1:-1] = (np.roll(c, 1, axis=1) + np.roll(c, -1, axis=1) + x[:-2] + x[2:] - 4 * c) / (h * h)
    return y


def apply_helmholtz(x: np.ndarray, beta) -> np.ndarray:
    """H x = x - beta * L_D x on interior rows, x on the wall rows."""
    return x - x.dtype.type(beta) * lap_dirichlet(x)


def solve_helmholtz(b: np.ndarray, beta) -> np.ndarray:
    """x with H x = b: wall rows x = b (the Dirichlet data), interior rows the
    exact solution of the linear system.  The x direction is periodic, so the
    discrete Fourier transform in x splits the system into one tridiagonal
    system in y per wavenumber k:
        (1 + 2s + 2s(1 - cos(2 pi k/N))) X_j - s (X_{j-1} + X_{j+1}) = B_j,
    j = 1..N-1, with the known wall values moved to the right-hand side;
    each is solved directly (banded LU)."""
    n = ops.n_of(b)
    s = float(beta) * n * n
    x = np.array(b, dtype=np.float64)
    if n < 2:
        return x
    rhs = np.array(b[1:-1], dtype=np.float64)
    rhs[0] += s * b[0]
    rhs[-1] += s * b[-1]
    rh = np.fft.fft(rhs, axis=1)
    k = np.arange(n)
    diag = 1.0 + 4.0 * s - 2.0 * s * np.cos(2.0 * np.pi * k / n)
    m = n - 1
    out = np.empty_like(rh)
    ab = np.zeros((3, m))
    for kk in range(n):
        ab[0, 1:] = -s
        ab[1, :] = diag[kk]
        ab[2, :-1] = -s
        out[:, kk] = solve_banded((1, 1), ab, rh[:, kk])
    x[1:-1] = np.real(np.fft.ifft(out, axis=1))
    return x


def advect_momentum(u: np.ndarray, v: np.ndarray):
    """((v.grad) u, (v.grad) v) = (u u_x + v u_y, u v_x + v v_y) by central
    differences (2h) on the interior rows (the y differences read the wall
    rows directly); zero on the wall rows."""
    n = ops.n_of(u)
    h = u.dtype.type(1) / n

    def dx(f):
        return (np.roll(f[1:-1], -1, axis=1) - np.roll(f[1:-1], 1, axis=1)) / (2 * h)

    def dy(f):
        return (f[2:] - f[:-2]) / (2 * h)

    au = np.zeros_like(u)
    av = np.zeros_like(v)
    au[1:-1] = u[1:-1] * dx(u) + v[1:-1] * dy(u)
    av[1:-1] = u[1:-1] * dx(v) + v[1:-1] * dy(v)
    return au, av


def predictor_rhs(u, v, dt, nu, theta, U):
    """Right-hand sides (bu, bv) of the two Helmholtz systems: the explicit
    part of eq. nopressmomentum on interior rows, the Dirichlet data on the
    wall rows (bu: 0 at the bottom, U at the top; bv: 0)."""
    au, av = advect_momentum(u, v)
    e = (1.0 - theta) * dt * nu
    bu = u - dt * au + e * lap_dirichlet(u)
    bv = v - dt * av + e * lap_dirichlet(v)
    bu[0] = 0.0
    bu[-1] = U
    bv[0] = 0.0
    bv[-1] = 0.0
    return bu, bv


def predict(u, v, dt=1e-4, nu=1.0, theta=0.5, U=1.0):
    """Provisional velocity (u*, v*) of eq. nopressmomentum."""
    bu, bv = predictor_rhs(u, v, dt, nu, theta, U)
    beta = theta * dt * nu
    return solve_helmholtz(bu, beta), solve_helmholtz(bv, beta)
