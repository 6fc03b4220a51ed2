"""Pins of the oracle's multigrid pieces (no GPU).

Restriction against the weighted adjoint of prolongation (assembled by
probing), interpolation order, the Chebyshev smoother against the closed-form
residual polynomial on Laplacian eigenmodes, symmetry/definiteness of the
V-cycle, and its contraction as a stationary iteration.
"""
import numpy as np
import pytest

from oracle import cg, dense, mg, ops, spectral


def _probe_rect(op, shape_in):
    size = shape_in[0] * shape_in[1]
    cols = []
    for k in range(size):
        e = np.zeros(size)
        e[k] = 1
        cols.append(op(e.reshape(shape_in)).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("nc", [4, 8])
def test_restriction_is_quarter_weighted_adjoint_of_prolongation(nc):
    nf = 2 * nc
    P = _probe_rect(mg.prolong, (nc + 1, nc))
    R = _probe_rect(mg.restrict, (nf + 1, nf))
    Wc = dense.weight_vector(nc)
    Wf = dense.weight_vector(nf)
    R_expect = 0.25 * (P.T * Wf[None, :]) / Wc[:, None]
    assert np.abs(R - R_expect).max() < 1e-15


def test_prolongation_reproduces_constants_and_injects():
    e = np.full((9, 8), 2.5)
    np.testing.assert_allclose(mg.prolong(e), 2.5, rtol=0, atol=1e-15)
    rng = np.random.default_rng(1)
    e = rng.standard_normal((9, 8))
    np.testing.assert_array_equal(mg.prolong(e)[0::2, 0::2], e)


def test_prolongation_fourth_order():
    """Cubic interpolation of cos(2 pi x) cos(pi y) (even across the walls):
    error falls ~16x per halving of h."""
    errs = []
    for nc in (8, 16, 32, 64):
        nf = 2 * nc
        f = lambda n: (np.cos(2 * np.pi * (np.arange(n) / n))[None, :]
                       * np.cos(np.pi * (np.arange(n + 1) / n))[:, None])
        errs.append(np.abs(mg.prolong(f(nc)) - f(nf)).max())
    for i in range(3):
        assert 14 < errs[i] / errs[i + 1] < 18


def test_restriction_of_smooth_field():
    """R preserves smooth fields to second order and constants exactly."""
    nf = 64
    r = np.full((nf + 1, nf), 1.5)
    np.testing.assert_allclose(mg.restrict(r), 1.5, atol=1e-15)
    errs = []
    for nf in (32, 64, 128):
        f = lambda n: (np.cos(2 * np.pi * (np.arange(n) / n))[None, :]
                       * np.cos(np.pi * (np.arange(n + 1) / n))[:, None])
        errs.append(np.abs(mg.restrict(f(nf)) - f(nf // 2)).max())
    assert errs[0] / errs[1] > 3.8 and errs[1] / errs[2] > 3.8


def test_chebyshev_coefficients_against_residual_polynomial():
    """With D constant (5-point Laplacian) the eigenmodes of D^{-1}A are the
    cosine modes; k Chebyshev steps from x = 0 leave the error
    T_k((theta - mu)/delta) / T_k(theta/delta) times the mode."""
    n = 16
    lev = mg.Level("lap", n, degree=3, ratio=4.0)
    lmax, lmin = 2.0, 0.5
    theta, delta = (lmax + lmin) / 2, (lmax - lmin) / 2
    T3 = lambda t: 4 * t ** 3 - 3 * t
    j = np.arange(n + 1)[:, None]
    i = np.arange(n)[None, :]
    for k, l in [(1, 1), (3, 5), (8, 16), (6, 2)]:
        mode = np.cos(2 * np.pi * k * i / n) * np.cos(np.pi * l * j / n)
        lam = spectral.lap_eigenvalue_full(n, k, l)
        mu = lam / (-4.0 * n * n)
        b = ops.lap5(mode)
        x = mg.smooth(lev, np.zeros_like(b), b)
        factor = T3((theta - mu) / delta) / T3(theta / delta)
        np.testing.assert_allclose(mode - x, factor * mode, atol=1e-12)


def test_jacobi_option_is_damped_jacobi():
    n = 16
    lev = mg.Level("lap", n, smoother="jacobi", degree=2)
    j = np.arange(n + 1)[:, None]
    i = np.arange(n)[None, :]
    mode = np.cos(2 * np.pi * 3 * i / n) * np.cos(np.pi * 4 * j / n)
    mu = spectral.lap_eigenvalue_full(n, 3, 4) / (-4.0 * n * n)
    b = ops.lap5(mode)
    x = mg.smooth(lev, np.zeros_like(b), b)
    np.testing.assert_allclose(mode - x, (1 - 0.8 * mu) ** 2 * mode, atol=1e-13)


@pytest.mark.parametrize("kind,c", [("ch", 1e-7), ("ch", 3e-4), ("lap", 0.0)])
def test_vcycle_is_weighted_symmetric_and_definite(kind, c):
    n = 32
    levels = mg.hierarchy(kind, n, c)
    rng = np.random.default_rng(7)
    r1 = rng.standard_normal((n + 1, n))
    r2 = rng.standard_normal((n + 1, n))
    if kind == "lap":
        r1 -= ops.wmean(r1)
        r2 -= ops.wmean(r2)
    a = ops.wdot(mg.vcycle(levels, r1), r2)
    b = ops.wdot(r1, mg.vcycle(levels, r2))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    q = ops.wdot(mg.vcycle(levels, r1), r1)
    assert q > 0 if kind == "ch" else q < 0


@pytest.mark.parametrize("kind,c,bound", [("ch", 1e-7, 0.5), ("ch", 1e-3, 0.5), ("lap", 0.0, 0.2)])
def test_vcycle_contraction(kind, c, bound):
    """x <- x + V(b - A x) converges to the exact solution at rate < bound."""
    n = 64
    levels = mg.hierarchy(kind, n, c)
    rng = np.random.default_rng(8)
    b = rng.standard_normal((n + 1, n))
    if kind == "lap":
        b -= ops.wmean(b)
        xs = spectral.solve_poisson(b)
        A = ops.lap5
    else:
        xs = spectral.solve_ch(b, c)
        A = lambda v: ops.apply_ch(v, c)
    x = np.zeros_like(b)
    errs = []
    for _ in range(6):
        x = x + mg.vcycle(levels, b - A(x))
        if kind == "lap":
            x = mg.project(x)
        errs.append(ops.wnorm(x - xs))
    rates = [errs[i + 1] / errs[i] for i in range(len(errs) - 1)]
    assert max(rates[1:]) < bound


def test_coarse_solve_exact():
    levels = mg.hierarchy("ch", 4, 2e-3)
    assert len(levels) == 1
    rng = np.random.default_rng(9)
    b = rng.standard_normal((5, 4))
    x = levels[0].coarse_solve(b)
    np.testing.assert_allclose(x, spectral.solve_ch(b, 2e-3), atol=1e-13)
    lp = mg.Level("lap", 4)
    p = lp.coarse_solve(b)
    np.testing.assert_allclose(p, spectral.solve_poisson(b), atol=1e-13)


def test_mg_pcg_reaches_spectral_solution():
    n = 64
    c = 1e-7
    levels = mg.hierarchy("ch", n, c)
    rng = np.random.default_rng(10)
    b = rng.standard_normal((n + 1, n))
    x, it, hist = cg.pcg(lambda v: ops.apply_ch(v, c), b,
                         precond=lambda r: mg.vcycle(levels, r), rtol=1e-12)
    assert it <= 12
    xs = spectral.solve_ch(b, c)
    assert ops.wnorm(x - xs) / ops.wnorm(xs) < 1e-12
