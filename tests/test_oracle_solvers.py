"""Pins of the oracle's solvers, chemical potential and step (no GPU).

Exact solves are checked against dense numpy.linalg.solve on tiny grids with
the explicitly assembled matrices (Sec. 4.1 row values + eq. discreteBC),
against closed-form eigenpairs, against plain weighted CG, and in long double.
The step is checked against invariants (mass conservation, constant state,
linearised amplification, divergence compatibility).
"""
import numpy as np
import pytest
import sympy

import synthetic as S
from oracle import cg, dense, fh, ops, spectral, step


# --------------------------------------------------------------- chemical potential
def test_mu_fh_is_symbolic_derivative_of_f_fh():
    p, N, chi = sympy.symbols("phi N chi", positive=True)
    f = (p / N) * sympy.log(p) + (1 - p) * sympy.log(1 - p) + chi * p * (1 - p)
    dfdp = sympy.lambdify((p, N, chi), sympy.diff(f, p), "numpy")
    phis = np.array([1e-6, 0.02, 0.3, 0.5, 0.9, 1 - 1e-6])
    np.testing.assert_allclose(fh.mu_fh(phis, 100.0, 0.6), dfdp(phis, 100.0, 0.6),
                               rtol=1e-13, atol=1e-13)


def test_mu_fh_central_difference_of_f_fh():
    phis = np.linspace(0.01, 0.95, 37)
    eps = 1e-6
    fd = (fh.f_fh(phis + eps, 100.0, 0.6) - fh.f_fh(phis - eps, 100.0, 0.6)) / (2 * eps)
    np.testing.assert_allclose(fh.mu_fh(phis, 100.0, 0.6), fd, atol=1e-8)


def test_mu_fh_value_at_half():
    # ln(1/2)/100 + 1/100 - ln(1/2) - 1 + 0.6*(1 - 1) by hand
    expect = np.log(0.5) / 100 + 0.01 - np.log(0.5) - 1
    assert fh.mu_fh(0.5, 100.0, 0.6) == pytest.approx(expect, rel=1e-15)


def test_rhs_constant_state_is_phi():
    phi = np.full((17, 16), 0.25)
    np.testing.assert_allclose(fh.rhs_ch(phi, 1e-4, 1.0, 100.0, 0.6), phi, rtol=0, atol=1e-15)


def test_clamp_leaves_phi_untouched_and_counts():
    phi = S.initial_phi(32)
    phi2 = phi.copy()
    phi2[3, 4] = 0.0
    phi2[5, 6] = 1.0
    assert fh.count_clamped(phi2) == 2
    b = fh.rhs_ch(phi2, 1e-4, 1.0, 100.0, 0.6)
    assert np.all(np.isfinite(b))


# --------------------------------------------------------------- exact solves
@pytest.mark.parametrize("c", [1e-7, 1e-4, 0.3])
def test_spectral_ch_matches_dense_n8(c):
    rng = np.random.default_rng(11)
    b = rng.standard_normal((9, 8))
    x = spectral.solve_ch(b, c)
    xd = dense.solve_ch_dense(b, c)
    assert np.abs(x - xd).max() <= 1e-13 * max(1.0, np.abs(xd).max())


def test_spectral_poisson_matches_bordered_dense_n8():
    rng = np.random.default_rng(12)
    rhs = rng.standard_normal((9, 8))
    p = spectral.solve_poisson(rhs)
    pd = dense.solve_poisson_dense(rhs)
    assert np.abs(p - pd).max() <= 1e-13 * np.abs(pd).max()
    assert abs(ops.wmean(p)) < 1e-15 * np.abs(p).max() * 100


@pytest.mark.parametrize("n,k,l", [(16, 2, 3), (32, 5, 0), (32, 0, 7)])
def test_spectral_poisson_on_eigenmode(n, k, l):
    j = np.arange(n + 1)[:, None]
    i = np.arange(n)[None, :]
    mode = np.cos(2 * np.pi * k * i / n) * np.cos(np.pi * l * j / n)
    lam = spectral.lap_eigenvalue_full(n, k, l)
    p = spectral.solve_poisson(mode)
    np.testing.assert_allclose(p, mode / lam, atol=1e-14 * np.abs(mode / lam).max())
    c = 2e-5
    x = spectral.solve_ch(mode, c)
    np.testing.assert_allclose(x, mode / (1 + c * lam * lam), atol=1e-14)


def test_spectral_poisson_constant_rhs_gives_zero():
    p = spectral.solve_poisson(np.full((17, 16), 3.0))
    assert np.abs(p).max() < 1e-13


def test_spectral_residuals_small():
    n = 128
    rng = np.random.default_rng(4)
    b = rng.standard_normal((n + 1, n))
    c = 1e-7
    x = spectral.solve_ch(b, c)
    assert ops.wnorm(b - ops.apply_ch(x, c)) / ops.wnorm(b) < 1e-13
    p = spectral.solve_poisson(b)
    f = b - ops.wmean(b)
    assert ops.wnorm(f - ops.lap5(p)) / ops.wnorm(f) < 1e-13


def test_long_double_agrees_with_float64():
    n = 64
    b = S.random_field(n, 9)
    c = 1e-7 * 10
    x64 = spectral.solve_ch(b, c)
    xld = spectral.solve_ch(b.astype(np.longdouble), c)
    assert xld.dtype == np.longdouble
    assert float(ops.wnorm(x64 - xld) / ops.wnorm(xld)) < 1e-14
    # the long-double residual, evaluated with the long-double stencil, is far below float64's
    r = b.astype(np.longdouble) - ops.apply_ch(xld, np.longdouble(c))
    assert float(ops.wnorm(r) / ops.wnorm(b.astype(np.longdouble))) < 1e-16


def test_spectral_matches_weighted_cg():
    n = 32
    rng = np.random.default_rng(2)
    b = rng.standard_normal((n + 1, n))
    c = 1e-5
    from oracle import mg
    diag = mg.ch_diagonal(n, c)
    x, it, hist = cg.pcg(lambda v: ops.apply_ch(v, c), b, precond=cg.jacobi_preconditioner(diag),
                         rtol=1e-13, maxit=5000)
    xs = spectral.solve_ch(b, c)
    assert ops.wnorm(x - xs) / ops.wnorm(xs) < 1e-11
    rhs = b - ops.wmean(b)
    p, it, hist = cg.pcg(ops.lap5, rhs, rtol=1e-13, maxit=5000, project=True)
    ps = spectral.solve_poisson(rhs)
    assert ops.wnorm(p - ps) / ops.wnorm(ps) < 1e-10


# --------------------------------------------------------------- step invariants
def test_step_conserves_mass():
    n = 64
    phi = S.initial_phi(n)
    u, v = S.inflow_velocity(n)
    m0 = ops.mass(phi)
    phi1 = phi
    for _ in range(5):
        phi1, p, uu, vv = step.step(phi1, u, v)
        assert abs(ops.mass(phi1) - m0) / m0 < 1e-13


def test_step_constant_state_fixed_point():
    n = 32
    phi = np.full((n + 1, n), 0.17)
    u = np.zeros((n + 1, n))
    phi1, p, uu, vv = step.step(phi, u, u)
    np.testing.assert_allclose(phi1, phi, rtol=0, atol=1e-15)
    assert np.abs(p).max() == 0


@pytest.mark.parametrize("k,l", [(1, 2), (3, 0), (5, 7)])
def test_step_linearised_amplification(k, l):
    """phi = phibar + eps*mode: one step multiplies the mode by
    (1 - dt M mu'(phibar) |lam|) / (1 + c lam^2) + O(eps)."""
    n, dt, M, kappa, Np, chi = 32, 1e-4, 1.0, 1e-3, 100.0, 0.6
    pb, eps = 0.2, 1e-7
    j = np.arange(n + 1)[:, None]
    i = np.arange(n)[None, :]
    mode = np.cos(2 * np.pi * k * i / n) * np.cos(np.pi * l * j / n)
    lam = spectral.lap_eigenvalue_full(n, k, l)
    mup = 1 / (Np * pb) + 1 / (1 - pb) - 2 * chi
    g = (1 + dt * M * mup * lam) / (1 + dt * M * kappa * lam * lam)
    phi1, *_ = step.step(pb + eps * mode, np.zeros((n + 1, n)), np.zeros((n + 1, n)),
                         dt=dt, M=M, kappa=kappa, Npoly=Np, chi=chi)
    amp = ops.wdot(phi1 - pb, mode) / ops.wdot(mode, mode) / eps
    assert amp == pytest.approx(g, rel=1e-5)


def test_pressure_rhs_compatible_and_velocity_update():
    n = 64
    u, v = S.inflow_velocity(n)
    dt = 1e-4
    rhs_raw = ops.divergence(u, v) / dt
    assert abs(ops.wmean(rhs_raw)) < 1e-9 * np.abs(rhs_raw).max()
    p, uu, vv = step.projection(u, v, dt)
    gx, gy = ops.gradient(p)
    np.testing.assert_allclose(uu, u - dt * gx, rtol=0, atol=1e-15)
    np.testing.assert_allclose(vv, v - dt * gy, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(vv[0], v[0])      # no normal flow correction on the walls
    # the spectral p solves L p = rhs
    rhs = step.pressure_rhs(u, v, dt)
    assert ops.wnorm(ops.lap5(p) - rhs) / ops.wnorm(rhs) < 1e-13


def test_initial_condition_recipe():
    n = 64
    phi = S.initial_phi(n)
    assert phi.shape == (65, 64)
    assert 0.3 - 0.005 <= phi[0, 0] <= 0.3 + 0.005          # base layer
    assert 0.02 - 0.005 <= phi[-1, 0] <= 0.02 + 0.005       # outside
    j, i = int(0.25 * n), n // 2                             # inside the protrusion
    assert 0.3 - 0.005 <= phi[j, i] <= 0.3 + 0.005
    assert np.array_equal(phi, S.initial_phi(n))            # seeded
