"""Pins of the oracle's grid operators against what the paper prints and what
the mathematics fixes (no GPU).

Paper: arXiv:1811.11842.  Laplacian row values and the wrap example come from
Sec. 4.1 (Listing "Constructing the matrix with DMDA" and the paragraph
after it), the ghost rules from Sec. 4, eq. discreteBC.
"""
import json
import os

import numpy as np
import pytest

from oracle import dense, ops, spectral

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_laplacian_row.json")


def _idx(n, i, j):
    return j * n + (i % n)


@pytest.fixture(scope="module")
def paper_row():
    with open(GOLD) as f:
        return json.load(f)


@pytest.mark.parametrize("n", [4, 8])
def test_lap5_interior_row_matches_paper_listing(paper_row, n):
    """Interior rows of -h^2 L carry exactly the listing's 4, -1, -1, -1, -1."""
    A = dense.probe(ops.lap5, n)
    h2 = 1.0 / (n * n)
    for j in range(1, n):
        for i in range(n):
            row = -h2 * A[_idx(n, i, j)]
            expect = np.zeros_like(row)
            for e in paper_row["row"]:
                expect[_idx(n, i + e["di"], j + e["dj"])] += e["value"]
            np.testing.assert_allclose(row, expect, atol=1e-12)


def test_lap5_periodic_wrap_example(paper_row):
    """Row i = 0: the neighbour i-1 = -1 sits in column nx-1 (Sec. 4.1)."""
    n = paper_row["example_domain"]["Nx"]
    A = dense.probe(ops.lap5, n)
    row = -A[_idx(n, 0, 2)] / (n * n)
    assert row[_idx(n, n - 1, 2)] == pytest.approx(-1.0)
    assert row[_idx(n, 1, 2)] == pytest.approx(-1.0)


@pytest.mark.parametrize("n", [4, 8])
def test_lap5_wall_rows_follow_reflection(n):
    """Ghost row -1 equals row 1 (eq. discreteBC), so the wall row of -h^2 L is
    4 (centre), -1 (i+-1), -2 (row 1); mirrored at j = N."""
    A = dense.probe(ops.lap5, n)
    for j, jn in ((0, 1), (n, n - 1)):
        for i in range(n):
            row = -A[_idx(n, i, j)] / (n * n)
            expect = np.zeros_like(row)
            expect[_idx(n, i, j)] = 4
            expect[_idx(n, i - 1, j)] += -1
            expect[_idx(n, i + 1, j)] += -1
            expect[_idx(n, i, jn)] += -2
            np.testing.assert_allclose(row, expect, atol=1e-12)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_lap5_probe_equals_explicit_assembly(n):
    np.testing.assert_allclose(dense.probe(ops.lap5, n), dense.lap_explicit(n),
                               rtol=0, atol=1e-9 * n * n)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_bih13_equals_laplacian_squared(n):
    """The directly written 13-point stencil equals L L with the two-layer
    reflection (eq. discreteBC); L comes from the explicit assembly."""
    L = dense.lap_explicit(n)
    B = dense.probe(ops.bih13, n)
    LL = L @ L
    assert np.abs(B - LL).max() <= 1e-14 * np.abs(LL).max()


def test_bih13_rows_closed_form():
    """Rows of h^4 L^2 derived by hand from the reflection rule: interior
    centre 20, axis -8, diagonal 2, distance-two 1; wall row j=0: 20 centre,
    -8 (i+-1, 0), -16 (i, 1), 4 (i+-1, 1), 2 (i, 2), 1 (i+-2, 0); row j=1 has
    centre 21 (the ghost at j=-1 is row 1)."""
    n = 8
    B = dense.probe(ops.bih13, n) / n ** 4
    i = 3
    r0 = B[_idx(n, i, 0)]
    exp0 = {(0, 0): 20, (1, 0): -8, (-1, 0): -8, (0, 1): -16, (1, 1): 4, (-1, 1): 4,
            (0, 2): 2, (2, 0): 1, (-2, 0): 1}
    e = np.zeros_like(r0)
    for (di, dj), v in exp0.items():
        e[_idx(n, i + di, dj)] += v
    np.testing.assert_allclose(r0, e, atol=1e-10)
    r1 = B[_idx(n, i, 1)]
    exp1 = {(0, 1): 21, (0, 0): -8, (1, 0): 2, (-1, 0): 2, (1, 1): -8, (-1, 1): -8,
            (2, 1): 1, (-2, 1): 1, (0, 2): -8, (1, 2): 2, (-1, 2): 2, (0, 3): 1}
    e = np.zeros_like(r1)
    for (di, dj), v in exp1.items():
        e[_idx(n, i + di, dj)] += v
    np.testing.assert_allclose(r1, e, atol=1e-10)
    for j in range(n + 1):
        expect = 21 if j in (1, n - 1) else 20
        assert B[_idx(n, 0, j), _idx(n, 0, j)] == pytest.approx(expect)


@pytest.mark.parametrize("n", [8, 16])
def test_weighted_self_adjointness(n):
    """W L and W L^2 are symmetric (trapezoid weights 1/2 on the wall rows);
    the plain matrices are not."""
    w = dense.weight_vector(n)
    for op in (ops.lap5, ops.bih13):
        A = dense.probe(op, n)
        WA = w[:, None] * A
        assert np.abs(WA - WA.T).max() <= 1e-13 * np.abs(A).max()
        assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()


@pytest.mark.parametrize("n,k,l", [(8, 3, 5), (16, 1, 0), (16, 0, 16), (32, 7, 11), (32, 16, 1)])
def test_eigenpairs_closed_form(n, k, l):
    """cos/sin(2 pi k i/N) cos(pi l j/N) are eigenvectors; lam(k,l) =
    -(4/h^2)(sin^2(pi k/N) + sin^2(pi l/(2N))); L^2 has lam^2."""
    j = np.arange(n + 1)[:, None]
    i = np.arange(n)[None, :]
    lam = spectral.lap_eigenvalue_full(n, k, l)
    for fx in (np.cos, np.sin):
        v = fx(2 * np.pi * k * i / n) * np.cos(np.pi * l * j / n)
        if not np.any(v):
            continue
        scale = np.abs(v).max()
        np.testing.assert_allclose(ops.lap5(v), lam * v, atol=1e-12 * abs(lam) * scale + 1e-9)
        np.testing.assert_allclose(ops.bih13(v), lam * lam * v,
                                   atol=1e-12 * lam * lam * scale + 1e-6)


def test_weighted_sums_vanish():
    """sum_W L x = 0 and sum_W L^2 x = 0 (discrete no-flux: mass conservation)."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((33, 32))
    one = np.ones_like(x)
    assert abs(ops.wdot(ops.lap5(x), one)) <= 1e-12 * 32 ** 2 * x.size
    assert abs(ops.wdot(ops.bih13(x), one)) <= 1e-12 * 32 ** 4 * x.size


def test_laplacian_second_order_convergence():
    """Manufactured cos(2 pi x) cos(pi y) (satisfies all odd-derivative wall
    conditions): the discrete eigenvalue approaches -(4 pi^2 + pi^2) as O(h^2)."""
    exact = -(4 + 1) * np.pi ** 2
    errs = []
    for n in (16, 32, 64, 128):
        y = (np.arange(n + 1) / n)[:, None]
        x = (np.arange(n) / n)[None, :]
        v = np.cos(2 * np.pi * x) * np.cos(np.pi * y)
        errs.append(np.abs(ops.lap5(v) - exact * v).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 3.9 < r < 4.1


def test_biharmonic_second_order_convergence():
    exact = ((4 + 1) * np.pi ** 2) ** 2
    errs = []
    for n in (16, 32, 64, 128):
        y = (np.arange(n + 1) / n)[:, None]
        x = (np.arange(n) / n)[None, :]
        v = np.cos(2 * np.pi * x) * np.cos(np.pi * y)
        errs.append(np.abs(ops.bih13(v) - exact * v).max())
    for i in range(3):
        assert 3.9 < errs[i] / errs[i + 1] < 4.1


def test_divergence_and_gradient_closed_forms():
    """Central differences (Sec. 4): div(sin 2 pi x, sin pi y) and grad of
    cos(2 pi x) cos(pi y) converge at second order; grad_y vanishes on the
    walls (p even), div uses v odd across the walls."""
    errs_d, errs_g = [], []
    for n in (32, 64, 128):
        y = (np.arange(n + 1) / n)[:, None] * np.ones((1, n))
        x = (np.arange(n) / n)[None, :] * np.ones((n + 1, 1))
        u = np.sin(2 * np.pi * x)
        v = np.sin(np.pi * y)
        v[0] = 0
        v[-1] = 0
        d = ops.divergence(u, v)
        de = 2 * np.pi * np.cos(2 * np.pi * x) + np.pi * np.cos(np.pi * y)
        errs_d.append(np.abs(d - de).max())
        p = np.cos(2 * np.pi * x) * np.cos(np.pi * y)
        gx, gy = ops.gradient(p)
        assert np.all(gy[0] == 0) and np.all(gy[-1] == 0)
        ge = -np.pi * np.cos(2 * np.pi * x) * np.sin(np.pi * y)
        errs_g.append(max(np.abs(gx + 2 * np.pi * np.sin(2 * np.pi * x) * np.cos(np.pi * y)).max(),
                          np.abs(gy - ge).max()))
    for e in (errs_d, errs_g):
        assert 3.8 < e[0] / e[1] < 4.2 and 3.8 < e[1] / e[2] < 4.2


def test_divergence_weighted_sum_is_zero():
    """sum_W div_h(u, v) = v_N - v_0 by telescoping, = 0 with zero wall rows."""
    rng = np.random.default_rng(3)
    n = 64
    u = rng.standard_normal((n + 1, n))
    v = rng.standard_normal((n + 1, n))
    v[0] = v[-1] = 0
    s = ops.wdot(ops.divergence(u, v), np.ones_like(u))
    assert abs(s) <= 1e-11 * n * np.abs(u).sum() / n


def test_weights_mean_and_mass():
    n = 16
    one = np.ones((n + 1, n))
    assert ops.wdot(one, one) == n * n
    assert ops.wmean(3.5 * one) == pytest.approx(3.5)
    assert ops.mass(one) == pytest.approx(1.0)
    y = (np.arange(n + 1) / n)[:, None] * np.ones((1, n))
    assert ops.mass(y) == pytest.approx(0.5)       # trapezoid rule exact on linears
