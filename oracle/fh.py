"""Flory-Huggins chemical potential and the Cahn-Hilliard right-hand side
(oracle; test infrastructure).

The paper lists the Flory-Huggins parameters chi and N (parameter table of
Sec. 5) and writes the network transport as the modified Cahn-Hilliard
equation (Sec. 2.2, eq. modCH).  The reduced step evaluated here keeps the
mobility constant (M), drops advection and production, and splits the
chemical potential into the bulk Flory-Huggins part, taken explicitly, and the
gradient-energy part -kappa*Delta(phi), taken implicitly:

    (I + dt*M*kappa*Delta_h^2) phi^{n+1} = phi^n + dt*M*Delta_h mu_FH(phi^n).

mu_FH is the derivative of the Flory-Huggins mixing energy density
    f_FH(phi) = (phi/N) ln(phi) + (1 - phi) ln(1 - phi) + chi*phi*(1 - phi).
"""
from __future__ import annotations

import numpy as np

from .ops import lap5


def f_fh(phi, Npoly, chi):
    """Flory-Huggins mixing energy density (per unit volume, dimensionless)."""
    return (phi / Npoly) * np.log(phi) + (1 - phi) * np.log1p(-phi) \
        + chi * phi * (1 - phi)


def mu_fh(phi, Npoly, chi):
    """d f_FH / d phi = ln(phi)/N + 1/N - ln(1-phi) - 1 + chi*(1 - 2 phi)."""
    return np.log(phi) / Npoly + 1 / Npoly - np.log(1 - phi) - 1 \
        + chi * (1 - 2 * phi)


def clamp(phi, lo, hi):
    """Keep the logarithms finite: mu is evaluated at clamp(phi, lo, hi); phi
    itself is never modified, so mass is unaffected."""
    return np.minimum(np.maximum(phi, lo), hi)


def rhs_ch(phi, dt, M, Npoly, chi, lo=1e-6, hi=1.0 - 1e-6):
    """b = phi + dt*M*L mu_FH(clamp(phi)); mu is even across the walls
    (grad(delta f / delta phi) . n = 0, Sec. 4), which lap5 realises."""
    mu = mu_fh(clamp(phi, lo, hi), Npoly, chi)
    return phi + dt * M * lap5(mu)


def count_clamped(phi, lo=1e-6, hi=1.0 - 1e-6) -> int:
    return int(np.count_nonzero((phi < lo) | (phi > hi)))
