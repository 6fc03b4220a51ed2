"""Pins of the momentum predictor (oracle/momentum.py) against facts fixed
outside it: a sparse system assembled node by node and factorised directly,
the closed-form eigenpairs of the Dirichlet 5-point Laplacian, second-order
convergence to a manufactured continuous solution, the exact discrete
harmonicity of a linear profile (plane Couette flow is a fixed point of the
predictor), and the Crank-Nicolson / backward-Euler amplification factors of
a decaying shear mode."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synthetic as S
from oracle import momentum as mom
from oracle import ops


def assembled(n, beta):
    """Matrix of the implicit operator, node by node: identity rows on the
    walls; 1 + 4s and -s (four neighbours, periodic in x) in the interior."""
    s = beta * n * n
    size = (n + 1) * n
    rows, cols, vals = [], [], []
    for j in range(n + 1):
        for i in range(n):
            k = j * n + i
            if j == 0 or j == n:
                rows.append(k); cols.append(k); vals.append(1.0)
                continue
            rows.append(k); cols.append(k); vals.append(1.0 + 4.0 * s)
            for jj, ii in ((j, (i - 1) % n), (j, (i + 1) % n), (j - 1, i), (j + 1, i)):
                rows.append(k); cols.append(jj * n + ii); vals.append(-s)
    return sp.csc_matrix((vals, (rows, cols)), shape=(size, size))


@pytest.mark.parametrize("n,beta", [(8, 1e-2), (16, 3e-3), (32, 1.0)])
def test_solve_matches_direct_sparse_solve(n, beta):
    rng = np.random.default_rng(n)
    b = rng.standard_normal((n + 1, n))
    x = mom.solve_helmholtz(b, beta)
    ref = spla.spsolve(assembled(n, beta), b.ravel()).reshape(n + 1, n)
    assert np.max(np.abs(x - ref)) <= 1e-12 * np.max(np.abs(ref))
    # and apply_helmholtz is that matrix
    assert np.allclose(mom.apply_helmholtz(x, beta).ravel(), assembled(n, beta) @ x.ravel(),
                       rtol=0, atol=1e-12 * np.max(np.abs(b)))


@pytest.mark.parametrize("k,m", [(0, 1), (1, 1), (3, 2), (5, 7)])
def test_eigenfunctions(k, m):
    """sin(m pi y) cos(2 pi k x) vanishes on both walls and is an eigenvector of
    L_D with eigenvalue -(4/h^2)(sin^2(pi k h) + sin^2(pi m h / 2))."""
    n, beta = 32, 2e-3
    Y, X = S.node_coords(n)
    e = np.sin(m * np.pi * Y) * np.cos(2 * np.pi * k * X)
    e[0] = 0.0
    e[-1] = 0.0
    lam = 4.0 * n * n * (np.sin(np.pi * k / n) ** 2 + np.sin(np.pi * m / (2 * n)) ** 2)
    x = mom.solve_helmholtz(e, beta)
    assert np.max(np.abs(x - e / (1.0 + beta * lam))) <= 1e-14
    assert np.max(np.abs(mom.lap_dirichlet(e) + lam * e)) <= 1e-9 * lam


def test_linear_profile_is_harmonic():
    n, U = 64, 0.7
    Y, _ = S.node_coords(n)
    g = U * Y
    assert np.max(np.abs(mom.lap_dirichlet(g))) <= 1e-10
    assert np.max(np.abs(mom.solve_helmholtz(g, 5e-3) - g)) <= 1e-14
    assert np.array_equal(mom.solve_helmholtz(g, 0.0), g)


def test_second_order_convergence():
    """u = U y + sin(pi y) sin(2 pi x) solves u - beta Lap u = f with
    f = U y + (1 + 5 pi^2 beta) sin(pi y) sin(2 pi x) and the wall data 0, U."""
    beta, U = 1e-2, 0.4
    errs = []
    for n in (16, 32, 64):
        Y, X = S.node_coords(n)
        exact = U * Y + np.sin(np.pi * Y) * np.sin(2 * np.pi * X)
        f = U * Y + (1 + 5 * np.pi ** 2 * beta) * np.sin(np.pi * Y) * np.sin(2 * np.pi * X)
        f[0] = 0.0
        f[-1] = U
        errs.append(np.max(np.abs(mom.solve_helmholtz(f, beta) - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.7 < r < 4.3 for r in ratios), ratios


def test_advection_second_order_and_uniform_flow():
    def fields(n):
        Y, X = S.node_coords(n)
        u = np.sin(2 * np.pi * X) * np.sin(np.pi * Y) + 0.5
        v = np.cos(2 * np.pi * X) * Y * (1 - Y)
        ux = 2 * np.pi * np.cos(2 * np.pi * X) * np.sin(np.pi * Y)
        uy = np.pi * np.sin(2 * np.pi * X) * np.cos(np.pi * Y)
        vx = -2 * np.pi * np.sin(2 * np.pi * X) * Y * (1 - Y)
        vy = np.cos(2 * np.pi * X) * (1 - 2 * Y)
        return u, v, u * ux + v * uy, u * vx + v * vy

    errs = []
    for n in (32, 64, 128):
        u, v, eu, ev = fields(n)
        au, av = mom.advect_momentum(u, v)
        errs.append(max(np.max(np.abs(au - eu)[1:-1]), np.max(np.abs(av - ev)[1:-1])))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.7 < r < 4.3 for r in ratios), ratios
    n = 16
    au, av = mom.advect_momentum(np.full((n + 1, n), 0.3), np.zeros((n + 1, n)))
    assert not au.any() and not av.any()


def test_couette_flow_is_a_fixed_point():
    """u = U y, v = 0: no advection (u_x = 0, v = 0) and L_D u = 0, so the
    predictor returns the same field for any theta, dt, nu."""
    n, U = 64, 0.1
    Y, _ = S.node_coords(n)
    for theta in (0.5, 1.0):
        us, vs = mom.predict(U * Y, np.zeros_like(Y), dt=1e-3, nu=2.0, theta=theta, U=U)
        assert np.max(np.abs(us - U * Y)) <= 1e-14
        assert np.max(np.abs(vs)) == 0.0


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_shear_mode_amplification(theta):
    """u = sin(m pi y), v = 0, U = 0: u* = g u with
    g = (1 - (1-theta) dt nu lam) / (1 + theta dt nu lam), lam = 4 n^2 sin^2(pi m/(2n))."""
    n, m, dt, nu = 64, 3, 1e-3, 0.5
    Y, _ = S.node_coords(n)
    u = np.sin(m * np.pi * Y)
    u[0] = 0.0
    u[-1] = 0.0
    lam = 4.0 * n * n * np.sin(np.pi * m / (2 * n)) ** 2
    g = (1 - (1 - theta) * dt * nu * lam) / (1 + theta * dt * nu * lam)
    us, vs = mom.predict(u, np.zeros_like(u), dt=dt, nu=nu, theta=theta, U=0.0)
    assert np.max(np.abs(us - g * u)) <= 1e-13
    assert not vs.any()


def test_wall_rows_carry_the_dirichlet_data():
    n = 16
    rng = np.random.default_rng(3)
    u = rng.standard_normal((n + 1, n))
    v = rng.standard_normal((n + 1, n))
    us, vs = mom.predict(u, v, dt=1e-3, nu=1.0, theta=0.5, U=0.25)
    assert np.all(us[0] == 0.0) and np.all(us[-1] == 0.25)
    assert np.all(vs[0] == 0.0) and np.all(vs[-1] == 0.0)
    assert ops.n_of(us) == n
