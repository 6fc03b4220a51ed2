"""Crank-Nicolson Cahn-Hilliard step with extrapolated chemical potential
(oracle; test infrastructure only).

The paper takes Crank-Nicolson for the linear terms and extrapolation for the
nonlinear ones to get second order in time (Sec. 4, the paragraph on the
discretisation).  For the reduced Cahn-Hilliard equation
d phi/dt = M L (mu_FH(phi) - kappa L phi) that reads

    (I + c/2 L^2) phi^{n+1} = (I - c/2 L^2) phi^n + dt*M*L mu_FH(clamp(phi*)),
    phi* = (3 phi^n - phi^{n-1}) / 2,   c = dt*M*kappa,

i.e. the operator of the semi-implicit step with c/2.  On the first step
(no phi^{n-1}) phi* = phi^n.
"""
from __future__ import annotations

from . import fh, ops, spectral


def rhs_cn(phi, phi_prev, dt, M, kappa, Npoly, chi, lo=1e-6, hi=1.0 - 1e-6):
    c = dt * M * kappa
    star = phi if phi_prev is None else 1.5 * phi - 0.5 * phi_prev
    mu = fh.mu_fh(fh.clamp(star, lo, hi), Npoly, chi)
    return ops.apply_ch(phi, -0.5 * c) + dt * M * ops.lap5(mu)


def step_cn(phi, phi_prev=None, dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6,
            phi_lo=1e-6, phi_hi=1.0 - 1e-6):
    """phi^{n+1} from phi^n and phi^{n-1} (None on the first step)."""
    b = rhs_cn(phi, phi_prev, dt, M, kappa, Npoly, chi, phi_lo, phi_hi)
    return spectral.solve_ch(b, 0.5 * dt * M * kappa)


def run_cn(phi0, steps, **prm):
    prev, phi = None, phi0
    for _ in range(steps):
        prev, phi = phi, step_cn(phi, prev, **prm)
    return phi
