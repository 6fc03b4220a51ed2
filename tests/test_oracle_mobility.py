"""Pins of the variable-mobility Cahn-Hilliard step (oracle/mobility.py):
reduction to the constant-mobility operators (whose spectral solve is pinned
elsewhere), W-self-adjointness and conservation of div_h(m grad_h .),
second-order convergence to div(m grad f) for smooth m and f, the direct
sparse LU against the refined iterative solve, and mass conservation of the
step."""
import numpy as np
import pytest

import synthetic as S
from oracle import fh, mobility as mob, ops, spectral

PRM = dict(dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6)


def rand_m(n, seed):
    rng = np.random.default_rng(seed)
    return 0.05 + rng.random((n + 1, n))


def test_constant_mobility_reduces_to_the_laplacian():
    n = 32
    rng = np.random.default_rng(1)
    f = rng.standard_normal((n + 1, n))
    assert np.allclose(mob.lap_mob(f, np.full_like(f, 1.0)), ops.lap5(f), rtol=0,
                       atol=1e-12 * np.abs(ops.lap5(f)).max())
    assert np.allclose(mob.lap_mob(f, np.full_like(f, 0.37)), 0.37 * ops.lap5(f), rtol=0,
                       atol=1e-12 * np.abs(ops.lap5(f)).max())


def test_self_adjoint_conservative_and_kills_constants():
    n = 32
    rng = np.random.default_rng(2)
    m = rand_m(n, 3)
    x, y = rng.standard_normal((2, n + 1, n))
    a, b = ops.wdot(x, mob.lap_mob(y, m)), ops.wdot(mob.lap_mob(x, m), y)
    assert abs(a - b) <= 1e-12 * abs(a)
    s = ops.wdot(mob.lap_mob(x, m), np.ones_like(x))
    assert abs(s) <= 1e-12 * np.abs(mob.lap_mob(x, m)).sum()
    assert np.abs(mob.lap_mob(np.full_like(x, 2.5), m)).max() <= 1e-9


def test_second_order_convergence():
    """m = 1 + 0.5 cos(2 pi x) cos(pi y), f = sin(2 pi x) cos(2 pi y) + cos(pi y):
    both have zero normal derivative at the walls, so the reflected grid
    operator approximates div(m grad f) to O(h^2) up to the wall rows."""
    errs = []
    for n in (32, 64, 128):
        Y, X = S.node_coords(n)
        m = 1 + 0.5 * np.cos(2 * np.pi * X) * np.cos(np.pi * Y)
        f = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + np.cos(np.pi * Y)
        mx = -np.pi * np.sin(2 * np.pi * X) * np.cos(np.pi * Y)
        my = -0.5 * np.pi * np.cos(2 * np.pi * X) * np.sin(np.pi * Y)
        fx = 2 * np.pi * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        fy = -2 * np.pi * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) - np.pi * np.sin(np.pi * Y)
        lap = (-4 * np.pi ** 2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
               - 4 * np.pi ** 2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
               - np.pi ** 2 * np.cos(np.pi * Y))
        exact = m * lap + mx * fx + my * fy
        errs.append(np.abs(mob.lap_mob(f, m) - exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.6 < r < 4.4 for r in ratios), ratios


def test_constant_mobility_solve_is_the_spectral_solve():
    n, c, M = 64, 1e-7, 0.8
    rng = np.random.default_rng(4)
    b = 0.3 + 0.01 * rng.standard_normal((n + 1, n))
    x = mob.solve(b, np.full_like(b, M), c)
    ref = spectral.solve_ch(b.astype(np.longdouble), np.longdouble(c) * np.longdouble(M))
    assert float(ops.wnorm(x - ref) / ops.wnorm(ref)) <= 1e-15


@pytest.mark.parametrize("n", [16, 32])
def test_direct_and_refined_solves_agree(n):
    c = 1e-4
    m = rand_m(n, n)
    rng = np.random.default_rng(n + 1)
    b = rng.standard_normal((n + 1, n))
    xd = mob.solve_direct(b, m, c)
    xi = mob.solve(b, m, c)
    assert float(ops.wnorm(xi.astype(np.float64) - xd) / ops.wnorm(xd)) <= 1e-12
    # the refined iterate's residual is at the long-double evaluation floor,
    # about u_ld * 64 c n^4 max(m) |x| (u_ld = 5.4e-20): far below float64
    r = b.astype(np.longdouble) - mob.apply_mob(xi, m.astype(np.longdouble), np.longdouble(c))
    assert float(ops.wnorm(r) / ops.wnorm(b)) <= 1e-16


def test_step_conserves_mass_and_reduces_to_constant_mobility():
    n = 32
    phi = S.initial_phi(n)
    new = mob.step_mob(phi, **PRM)
    assert abs(float(ops.mass(new) - ops.mass(phi))) <= 1e-15 * float(ops.mass(phi))
    # where the mobility is constant the step is the constant-mobility one:
    # a uniform field stays uniform; and m = M everywhere gives fh.rhs_ch
    u = np.full((n + 1, n), 0.25)
    assert np.abs(mob.step_mob(u, **PRM) - 0.25).max() <= 1e-15
    b = mob.rhs_mob(phi, PRM["dt"], PRM["M"], PRM["Npoly"], PRM["chi"])
    p = fh.clamp(phi, 1e-6, 1 - 1e-6)
    mu = fh.mu_fh(p, PRM["Npoly"], PRM["chi"])
    assert np.allclose(b, phi + PRM["dt"] * mob.lap_mob(mu, PRM["M"] * p))
