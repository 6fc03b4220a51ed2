"""One time step of the reduced biofilm-flow model (oracle; test infrastructure).

  1. Cahn-Hilliard (Sec. 2.2 eq. modCH, constant mobility, no advection or
     production): b = phi + dt*M*L mu_FH(phi);  (I + dt*M*kappa*L^2) phi' = b.
  2. Pressure projection (Sec. 4: Chorin's method, eqs. pressuresolve and
     velocityupdate): rhs = div_h(u*)/dt with its weighted mean removed
     (null-space removal, Sec. 4.1), L p = rhs, weighted-mean-zero p, then
     v = u* - dt grad_h p.

Sign and scale of the pressure: the paper writes -div(grad p / rho) = div u and
v = u + grad p / rho; with rho = 1 (equal network and solvent densities in
the parameter table) the pressure used here is p = -p_paper / dt, which gives
the same corrected velocity.

Both solves use the exact spectral solver, so the result is the exact
solution of the discrete step (up to rounding in the chosen dtype).
"""
from __future__ import annotations

import numpy as np

from . import fh, ops, spectral


def step(phi, ustar, vstar, dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6,
         phi_lo=1e-6, phi_hi=1.0 - 1e-6):
    """Returns (phi_new, p, u, v)."""
    b = fh.rhs_ch(phi, dt, M, Npoly, chi, phi_lo, phi_hi)
    phi_new = spectral.solve_ch(b, dt * M * kappa)
    p, u, v = projection(ustar, vstar, dt)
    return phi_new, p, u, v


def pressure_rhs(ustar, vstar, dt):
    rhs = ops.divergence(ustar, vstar) / dt
    return rhs - ops.wmean(rhs)


def projection(ustar, vstar, dt):
    p = spectral.solve_poisson(pressure_rhs(ustar, vstar, dt))
    gx, gy = ops.gradient(p)
    return p, ustar - dt * gx, vstar - dt * gy


def run(phi0, ustar, vstar, steps, **params):
    """Several steps with u* held fixed (returns phi, p, u, v of the last)."""
    phi = phi0
    p = u = v = None
    for _ in range(steps):
        phi, p, u, v = step(phi, ustar, vstar, **params)
    return phi, p, u, v
