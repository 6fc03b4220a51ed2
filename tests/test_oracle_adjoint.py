"""Pins of the oracle's adjoint (oracle/adjoint.py) against what mathematics
fixes: transposes by dot-product identities and by probing, the derivative of
mu_FH by finite differences, and the whole rollout gradient by central finite
differences of the forward rollout (epsilon = 1e-6, as for the GPU check)."""
import numpy as np
import pytest

import synthetic as S
from oracle import adjoint as adj
from oracle import fh, ops, spectral

PRM = dict(dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6)


def _rand(n, seed):
    return np.random.default_rng(seed).standard_normal((n + 1, n))


@pytest.mark.parametrize("n", [8, 16])
def test_advect_transpose_dot_identity(n):
    phi, eta, u, v = (_rand(n, s) for s in (1, 2, 3, 4))
    lhs = np.sum(adj.advect(phi, u, v) * eta)
    rhs = np.sum(phi * adj.advect_T(eta, u, v))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(adj.advect(phi, u, v) * eta))


def test_advect_transpose_by_probing():
    """Assemble D column by column (unit vectors) and compare D^T with advect_T
    applied to unit vectors, entry by entry."""
    n = 4
    u, v = _rand(n, 5), _rand(n, 6)
    N = (n + 1) * n
    D = np.zeros((N, N))
    E = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        D[:, k] = adj.advect(e.reshape(n + 1, n), u, v).ravel()
        E[:, k] = adj.advect_T(e.reshape(n + 1, n), u, v).ravel()
    assert np.allclose(D.T, E, rtol=0, atol=1e-12)


def test_advect_of_constant_is_divergence():
    """D(1; u, v) = div_h(u, v) (constant phi), and D(phi; 0, 0) = 0."""
    n = 16
    u, v = _rand(n, 7), _rand(n, 8)
    assert np.allclose(adj.advect(np.ones((n + 1, n)), u, v), ops.divergence(u, v),
                       rtol=0, atol=1e-12)
    assert np.all(adj.advect(_rand(n, 9), np.zeros((n + 1, n)), np.zeros((n + 1, n))) == 0)


@pytest.mark.parametrize("n", [8, 32])
def test_lap_transpose_dot_identity(n):
    x, y = _rand(n, 10), _rand(n, 11)
    lhs = np.sum(ops.lap5(x) * y)
    rhs = np.sum(x * adj.lap_T(y))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(ops.lap5(x) * y))


def test_transpose_solve_dot_identity():
    n = 32
    c = 3e-6
    x, y = _rand(n, 12), _rand(n, 13)
    lhs = np.sum(spectral.solve_ch(x, c) * y)
    rhs = np.sum(x * adj.solve_ch_T(y, c))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # and A^T eta = lam with A applied as a matrix: sum(A e_k * eta) = lam_k
    eta = adj.solve_ch_T(y, c)
    n2 = (n + 1) * n
    k = np.random.default_rng(0).integers(0, n2, size=20)
    for kk in k:
        e = np.zeros(n2)
        e[kk] = 1.0
        col = ops.apply_ch(e.reshape(n + 1, n), c).ravel()
        assert abs(col @ eta.ravel() - y.ravel()[kk]) <= 1e-10 * np.abs(y).max()


def test_dmu_matches_finite_difference():
    phi = np.linspace(0.01, 0.95, 50)
    eps = 1e-6
    fd = (fh.mu_fh(phi + eps, 100.0, 0.6) - fh.mu_fh(phi - eps, 100.0, 0.6)) / (2 * eps)
    assert np.allclose(adj.dmu_fh(phi, 100.0, 0.6), fd, rtol=1e-7)


def test_objective_is_upper_half_integral():
    """J of phi = 1 is the area of the upper half (1/2); of phi = y it is
    int_{1/2}^1 y dy = 3/8 exactly (trapezoid rule is exact for linears)."""
    n = 16
    Y, _ = S.node_coords(n)
    assert abs(adj.objective(np.ones((n + 1, n))) - 0.5) <= 1e-15
    assert abs(adj.objective(Y.copy()) - 0.375) <= 1e-15


def _setup(n, U=1.0):
    phi0 = S.initial_phi(n)
    Y, _ = S.node_coords(n)
    base = Y * (2.0 - Y)
    u0, v0 = S.inflow_velocity(n, U=0.0)    # the noise only
    return phi0, base, u0, v0


def _J(phi0, U, chi, steps, noise_u, noise_v, base):
    n = ops.n_of(phi0)
    prm = dict(PRM, chi=chi)
    u, v, _, _ = adj.velocity(n, U, prm["dt"], noise_u, noise_v, base)
    return adj.objective(adj.rollout(phi0, u, v, steps, **prm))


@pytest.mark.parametrize("n,steps", [(16, 4), (32, 3)])
def test_rollout_gradient_matches_central_differences(n, steps):
    """Central differences of the forward rollout.  Their error is the
    truncation O(eps^2) plus the rounding of J (about 1e-17 absolute: J is
    about 1e-2 and the spectral solves are exact to rounding) divided by eps.
    dJ/dchi (1e-7 .. 4e-6) and dJ/dU (about 1e-11) are small, so they take
    eps = 1e-4 (noise 1e-13, truncation below 1e-9 relative); directional
    derivatives in phi0 (about 7e-2) take eps = 1e-6."""
    phi0, base, nu, nv = _setup(n)
    U, chi = 1.0, PRM["chi"]
    prm = dict(PRM)
    J, gphi, gchi, gU = adj.rollout_grad(phi0, U, steps, nu, nv, base, **prm)
    assert abs(J - _J(phi0, U, chi, steps, nu, nv, base)) <= 1e-15
    e = 1e-4
    fd_chi = (_J(phi0, U, chi + e, steps, nu, nv, base)
              - _J(phi0, U, chi - e, steps, nu, nv, base)) / (2 * e)
    assert abs(gchi - fd_chi) <= 1e-6 * abs(fd_chi)
    fd_U = (_J(phi0, U + e, chi, steps, nu, nv, base)
            - _J(phi0, U - e, chi, steps, nu, nv, base)) / (2 * e)
    assert abs(gU - fd_U) <= 1e-6 * abs(fd_U) + 1e-13
    assert gU != 0.0
    rng = np.random.default_rng(99)
    eps = 1e-6
    for _ in range(3):
        d = rng.standard_normal(phi0.shape)
        fd = (_J(phi0 + eps * d, U, chi, steps, nu, nv, base)
              - _J(phi0 - eps * d, U, chi, steps, nu, nv, base)) / (2 * eps)
        assert abs(np.sum(gphi * d) - fd) <= 1e-6 * abs(fd)


def test_a_planted_sign_error_is_caught():
    """The finite-difference check is sharp enough to see a wrong sign of the
    advective term in the adjoint (a plausible slip)."""
    n, steps = 16, 3
    phi0, base, nu, nv = _setup(n)
    prm = dict(PRM)
    good = adj.rollout_grad(phi0, 1.0, steps, nu, nv, base, **prm)
    orig = adj.advect_T
    try:
        adj.advect_T = lambda eta, u, v: -orig(eta, u, v)
        bad = adj.rollout_grad(phi0, 1.0, steps, nu, nv, base, **prm)
    finally:
        adj.advect_T = orig
    d = np.random.default_rng(5).standard_normal(phi0.shape)
    eps = 1e-6
    fd = (_J(phi0 + eps * d, 1.0, prm["chi"], steps, nu, nv, base)
          - _J(phi0 - eps * d, 1.0, prm["chi"], steps, nu, nv, base)) / (2 * eps)
    assert abs(np.sum(good[1] * d) - fd) <= 1e-6 * abs(fd)
    assert abs(np.sum(bad[1] * d) - fd) > 1e-6 * abs(fd)


def test_no_advection_means_no_inflow_sensitivity():
    """With zero velocity the step does not see U: the U gradient of the
    adjoint step vanishes, and the phi gradient is that of the plain step."""
    n = 16
    phi0 = S.initial_phi(n)
    z = np.zeros_like(phi0)
    lam = adj.objective_weights(n)
    l1, gc1, gu1 = adj.adjoint_step(phi0, z, z, z, z, lam, **PRM)
    l2, gc2, gu2 = adj.adjoint_step(phi0, None, None, None, None, lam, **PRM)
    assert gu1 == 0.0 and gu2 == 0.0
    assert np.array_equal(l1, l2) and gc1 == gc2
