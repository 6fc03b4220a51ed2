"""Adjoint of the Cahn-Hilliard rollout with advection (oracle; test
infrastructure only).

Forward map.  The paper's Cahn-Hilliard equation (Sec. 2.2, eq. modCH) carries
the advective flux div(phi v) of the network volume fraction.  The reduced
step keeps it explicit, with the velocity v = (u, v) of the projection step
(Sec. 4, eqs. pressuresolve and velocityupdate) held fixed over a rollout:

    b(phi)  = phi + dt*M*L mu_FH(clamp(phi)) - dt*D(phi; u, v),
    D(phi; u, v) = div_h(phi*u, phi*v)        (central, v odd across the walls)
    A phi'  = b(phi),  A = I + c L^2,  c = dt*M*kappa.

The velocity is the projection of the provisional field
u* = U*y*(2 - y) + noise_u, v* = noise_v, so it is linear in the inflow
speed U, with d(u, v)/dU = projection of (y*(2 - y), 0).

Objective ("detached biofilm mass"): J = integral of phi^N over y >= 1/2 by
the trapezoid rule, J = h^2 * sum_{i,j} W_j m_j phi^N_ij with m_j = 1 above
the middle row, 1/2 on it, 0 below.

Adjoint (plain transposes, Euclidean inner product):

    lam^N      = dJ/dphi^N = h^2 W m,
    eta        = A^{-T} lam^{n+1},  A^T = W A W^{-1} (A is self-adjoint in the
                 trapezoid inner product, so the transpose solve is the same
                 solve between two diagonal scalings),
    lam^n      = eta + dt*M*mu'(phi^n) * (L^T eta) - dt*D^T eta,  L^T = W L W^{-1},
    dJ/dchi   += dt*M * <L^T eta, 1 - 2*clamp(phi^n)>,
    dJ/dU     += -dt * <eta, D(phi^n; du, dv)>,
    dJ/dphi^0  = lam^0.

mu' is zero where the clamp is active (the clamp's derivative).  The
transposes are written out below and pinned by dot-product identities and by
central finite differences of the whole rollout (tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import numpy as np

from . import fh, ops, spectral, step as stepmod


def dmu_fh(phi, Npoly, chi):
    """d mu_FH / d phi = 1/(N phi) + 1/(1 - phi) - 2 chi (derivative of the
    Flory-Huggins chemical potential, Sec. 2.2)."""
    return 1.0 / (Npoly * phi) + 1.0 / (1.0 - phi) - 2.0 * chi


def advect(phi, u, v):
    """D(phi; u, v) = div_h(phi u, phi v): the explicit advective flux of
    eq. modCH with central differences (Sec. 4); phi is even and v odd across
    the walls, so phi*v is odd, as ops.divergence assumes for its second
    argument."""
    return ops.divergence(phi * u, phi * v)


def advect_T(eta, u, v):
    """Transpose of phi -> D(phi; u, v) for fixed (u, v).

    x part: (D_x phi)_i = (u_{i+1} phi_{i+1} - u_{i-1} phi_{i-1})/(2h), so
    (D_x^T eta)_k = u_k (eta_{k-1} - eta_{k+1})/(2h).
    y part: rows 1..N-1 use (v phi)_{j+1} - (v phi)_{j-1} over 2h; the wall rows
    fold the odd ghost onto the first interior row: row 0 is (v phi)_1 / h and
    row N is -(v phi)_{N-1} / h.  Collecting the coefficient of phi_{k,l}:
    (D_y^T eta)_l = v_l [em_l - ep_l] with
      em_l = eta_{l-1}/(2h) for l >= 2, eta_0/h for l = 1, 0 for l = 0;
      ep_l = eta_{l+1}/(2h) for l <= N-2, eta_N/h for l = N-1, 0 for l = N.
    """
    n = ops.n_of(eta)
    h = eta.dtype.type(1) / n
    dx = u * (np.roll(eta, 1, axis=1) - np.roll(eta, -1, axis=1)) / (2 * h)
    em = np.zeros_like(eta)
    ep = np.zeros_like(eta)
    em[2:] = eta[1:-1] / (2 * h)
    em[1] = eta[0] / h
    ep[:-2] = eta[1:-1] / (2 * h)
    ep[-2] = eta[-1] / h
    return dx + v * (em - ep)


def lap_T(eta):
    """L^T = W L W^{-1} (L is self-adjoint in the trapezoid inner product)."""
    w = ops.weights(ops.n_of(eta), eta.dtype)
    return w * ops.lap5(eta / w)


def solve_ch_T(lam, c):
    """eta = A^{-T} lam = W A^{-1} (W^{-1} lam) with the exact spectral solve."""
    w = ops.weights(ops.n_of(lam), lam.dtype)
    return w * spectral.solve_ch(lam / w, c)


def rhs_adv(phi, u, v, dt, M, Npoly, chi, lo=1e-6, hi=1.0 - 1e-6):
    """b(phi) = phi + dt*M*L mu_FH(clamp(phi)) - dt*D(phi; u, v)."""
    b = fh.rhs_ch(phi, dt, M, Npoly, chi, lo, hi)
    if u is not None:
        b = b - dt * advect(phi, u, v)
    return b


def step_adv(phi, u, v, dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6,
             phi_lo=1e-6, phi_hi=1.0 - 1e-6):
    """One Cahn-Hilliard step with explicit advection by the fixed (u, v)."""
    b = rhs_adv(phi, u, v, dt, M, Npoly, chi, phi_lo, phi_hi)
    return spectral.solve_ch(b, dt * M * kappa)


def adjoint_step(phi, u, v, du, dv, lam, dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0,
                 chi=0.6, phi_lo=1e-6, phi_hi=1.0 - 1e-6):
    """(lam^n, dJ/dchi contribution, dJ/dU contribution) from lam^{n+1}.

    du, dv: the direction d(u, v)/dU (None: no U contribution)."""
    c = dt * M * kappa
    eta = solve_ch_T(lam, c)
    lt = lap_T(eta)
    phat = fh.clamp(phi, phi_lo, phi_hi)
    active = (phi >= phi_lo) & (phi <= phi_hi)
    mup = np.where(active, dmu_fh(phat, Npoly, chi), 0.0)
    lam_prev = eta + dt * M * mup * lt
    if u is not None:
        lam_prev = lam_prev - dt * advect_T(eta, u, v)
    g_chi = dt * M * float(np.sum(lt * (1.0 - 2.0 * phat)))
    g_u = 0.0
    if du is not None:
        g_u = -dt * float(np.sum(eta * advect(phi, du, dv)))
    return lam_prev, g_chi, g_u


def objective_weights(n, dtype=np.float64):
    """h^2 W_j m_j: dJ/dphi of J = integral of phi over y >= 1/2 (n even)."""
    h = 1.0 / n
    m = np.zeros((n + 1, 1), dtype=dtype)
    m[n // 2 + 1:] = 1.0
    m[n // 2] = 0.5
    return (h * h) * ops.weights(n, dtype) * m * np.ones((1, n), dtype=dtype)


def objective(phi):
    return float(np.sum(objective_weights(ops.n_of(phi), phi.dtype) * phi))


def velocity(n, U, dt, noise_u, noise_v, base):
    """Projected velocity of u* = U*base + noise_u, v* = noise_v, and its
    derivative with respect to U (projection of (base, 0))."""
    _, u, v = stepmod.projection(U * base + noise_u, noise_v, dt)
    _, du, dv = stepmod.projection(base, np.zeros_like(base), dt)
    return u, v, du, dv


def rollout(phi0, u, v, steps, **prm):
    phi = phi0
    for _ in range(steps):
        phi = step_adv(phi, u, v, **prm)
    return phi


def rollout_grad(phi0, U, steps, noise_u, noise_v, base, dt=1e-4, M=1.0, kappa=1e-3,
                 Npoly=100.0, chi=0.6, phi_lo=1e-6, phi_hi=1.0 - 1e-6):
    """J, dJ/dphi0, dJ/dchi, dJ/dU of the rollout (all states kept)."""
    n = ops.n_of(phi0)
    prm = dict(dt=dt, M=M, kappa=kappa, Npoly=Npoly, chi=chi, phi_lo=phi_lo,
               phi_hi=phi_hi)
    u, v, du, dv = velocity(n, U, dt, noise_u, noise_v, base)
    states = [phi0]
    for _ in range(steps):
        states.append(step_adv(states[-1], u, v, **prm))
    J = objective(states[-1])
    lam = objective_weights(n, phi0.dtype)
    g_chi = g_u = 0.0
    for k in range(steps - 1, -1, -1):
        lam, gc, gu = adjoint_step(states[k], u, v, du, dv, lam, **prm)
        g_chi += gc
        g_u += gu
    return J, lam, g_chi, g_u
