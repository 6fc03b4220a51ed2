"""Pins of the Crank-Nicolson step (oracle/cn.py): second order in time
(against the first-order semi-implicit step, which the same check shows to
be first order), mass conservation, and the reduction to the explicit step
when kappa = 0."""
import numpy as np

import synthetic as S
from oracle import cn, fh, ops, spectral

PRM = dict(M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6)


def smooth_phi(n):
    Y, X = S.node_coords(n)
    return 0.3 + 0.05 * np.cos(2 * np.pi * X) * np.cos(np.pi * Y) \
        + 0.03 * np.cos(4 * np.pi * X + 0.3) * np.cos(2 * np.pi * Y)


def euler_run(phi0, steps, dt):
    phi = phi0
    for _ in range(steps):
        b = fh.rhs_ch(phi, dt, PRM["M"], PRM["Npoly"], PRM["chi"])
        phi = spectral.solve_ch(b, dt * PRM["M"] * PRM["kappa"])
    return phi


def test_second_order_in_time():
    """Error at T = 8e-3 against a reference with 64x smaller steps: halving
    dt divides the CN error by about 4 (the semi-implicit Euler error by 2).
    The first CN step uses phi* = phi^n (first order locally, second order
    globally since it happens once)."""
    n, T = 16, 8e-3
    phi0 = smooth_phi(n)
    ref = cn.run_cn(phi0, 512, dt=T / 512, **PRM)
    errs_cn, errs_eu = [], []
    for steps in (8, 16, 32):
        dt = T / steps
        errs_cn.append(ops.wnorm(cn.run_cn(phi0, steps, dt=dt, **PRM) - ref))
        errs_eu.append(ops.wnorm(euler_run(phi0, steps, dt) - ref))
    r_cn = [errs_cn[k] / errs_cn[k + 1] for k in range(2)]
    r_eu = [errs_eu[k] / errs_eu[k + 1] for k in range(2)]
    assert all(3.5 < r < 4.6 for r in r_cn), r_cn
    assert all(1.7 < r < 2.3 for r in r_eu), r_eu


def test_mass_conserved():
    n = 32
    phi0 = S.initial_phi(n)
    phi1 = cn.step_cn(phi0, None, dt=1e-4, **PRM)
    phi2 = cn.step_cn(phi1, phi0, dt=1e-4, **PRM)
    m0 = ops.mass(phi0)
    assert abs(ops.mass(phi1) - m0) <= 1e-13 * m0
    assert abs(ops.mass(phi2) - m0) <= 1e-13 * m0


def test_kappa_zero_is_explicit_step():
    """kappa = 0: no implicit part, phi' = phi + dt M L mu(phi*)."""
    n = 16
    phi0 = S.initial_phi(n)
    prev = phi0 + 1e-3 * S.random_field(n, 3)
    got = cn.step_cn(phi0, prev, dt=1e-5, M=1.0, kappa=0.0, Npoly=100.0, chi=0.6)
    star = 1.5 * phi0 - 0.5 * prev
    want = phi0 + 1e-5 * ops.lap5(fh.mu_fh(star, 100.0, 0.6))
    assert np.allclose(got, want, rtol=0, atol=1e-14)
