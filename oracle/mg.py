"""Geometric multigrid V-cycle for the two grid operators, written plainly
(oracle; test infrastructure).

The paper solves with Krylov + Jacobi and names better preconditioners as
future work (Sec. 4.1, Sec. 6).  The preconditioner here is a standard
vertex-centred geometric V-cycle whose smoother is Jacobi-based:

  * level l has N_l = N / 2^l intervals, h_l = 1/N_l, shape (N_l+1, N_l); the
    operator is re-discretised on every level (Laplacian L_l, or I + c L_l^2
    with the same c);
  * smoother: a Chebyshev polynomial in D^{-1} A of degree k (Chebyshev
    acceleration of Jacobi; k = 1 is damped Jacobi with weight 1/theta), or
    plain damped Jacobi with weight omega;
  * prolongation: tensor-product cubic interpolation (weights -1/16, 9/16,
    9/16, -1/16 at the odd fine nodes), periodic in x, even reflection in y;
  * restriction: R = (1/4) W_c^{-1} P^T W_f, the weighted adjoint of P, which is
    the 7x7 stencil with per-direction weights {0: 1/2, +-1: 9/32, +-3: -1/32}
    on the evenly reflected fine field;
  * coarsest grid N_l = 4: exact dense solve (for the Laplacian with the
    weighted-mean constraint).

Cubic transfers: for a fourth-order operator the orders of the transfers
must satisfy m_P + m_R > 4 for level-independent convergence; bilinear
interpolation with full weighting (2 + 2) does not.

Chebyshev interval: [lmax/ratio, lmax] with lmax the Gershgorin bound of
D^{-1} A: 2 for the 5-point Laplacian; (1 + 64 s)/(1 + 20 s), s = c N_l^4, for
the Cahn-Hilliard operator.
"""
from __future__ import annotations

import numpy as np

from . import dense
from .ops import apply_ch, lap5, n_of, wmean

COARSEST = 4


def ch_diagonal(n: int, c) -> np.ndarray:
    """Diagonal of I + c L^2 with reflection: 1 + s*20, and 1 + s*21 on rows
    j = 1 and j = N-1 (the reflected ghost at distance 2 lands on the centre)."""
    s = c * float(n) ** 4
    d = np.full((n + 1, n), 1 + 20 * s)
    d[1, :] = 1 + 21 * s
    d[n - 1, :] = 1 + 21 * s
    return d


def lap_diagonal(n: int) -> np.ndarray:
    return np.full((n + 1, n), -4.0 * n * n)


def ch_lmax(n: int, c) -> float:
    s = c * float(n) ** 4
    return (1 + 64 * s) / (1 + 20 * s)


LAP_LMAX = 2.0


def chebyshev_coefficients(lmax: float, ratio: float, degree: int):
    """Coefficients (a_k, g_k) of the three-term Chebyshev iteration on
    [lmax/ratio, lmax] (Saad, Iterative Methods for Sparse Linear Systems,
    Sec. 12.3.2):
        x_{k+1} = x_k + a_k D^{-1}(b - A x_k) + g_k (x_k - x_{k-1}).
    With theta = (lmax + lmin)/2, delta = (lmax - lmin)/2, sigma = theta/delta:
    a_0 = 1/theta, g_0 = 0; rho_0 = 1/sigma, rho_k = 1/(2 sigma - rho_{k-1}),
    a_k = 2 rho_k / delta, g_k = rho_k rho_{k-1}."""
    lmin = lmax / ratio
    theta = (lmax + lmin) / 2
    delta = (lmax - lmin) / 2
    sigma = theta / delta
    a = [1 / theta]
    g = [0.0]
    rho = 1 / sigma
    for _ in range(1, degree):
        rho_new = 1 / (2 * sigma - rho)
        a.append(2 * rho_new / delta)
        g.append(rho_new * rho)
        rho = rho_new
    return a, g


def _ys(x: np.ndarray, d: int) -> np.ndarray:
    """Row j+d of an (m+1)-row array, even reflection at rows 0 and m."""
    m = x.shape[0] - 1
    j = np.arange(m + 1) + d
    j = np.where(j < 0, -j, j)
    j = np.where(j > m, 2 * m - j, j)
    return x[j]


def prolong(e: np.ndarray) -> np.ndarray:
    """Cubic interpolation from (Nc+1, Nc) to (2Nc+1, 2Nc)."""
    nc = n_of(e)
    t = np.zeros((nc + 1, 2 * nc), dtype=e.dtype)
    t[:, 0::2] = e
    t[:, 1::2] = (-np.roll(e, 1, axis=1) + 9 * e + 9 * np.roll(e, -1, axis=1)
                  - np.roll(e, -2, axis=1)) / 16
    f = np.zeros((2 * nc + 1, 2 * nc), dtype=e.dtype)
    f[0::2] = t
    f[1::2] = ((-_ys(t, -1) + 9 * t + 9 * _ys(t, 1) - _ys(t, 2)) / 16)[:-1]
    return f


RESTRICT_W = {0: 0.5, 1: 9 / 32, -1: 9 / 32, 3: -1 / 32, -3: -1 / 32}


def restrict(r: np.ndarray) -> np.ndarray:
    """(1/4) W_c^{-1} P^T W_f r, as a stencil on the evenly reflected fine field."""
    out = np.zeros_like(r)
    for dj, wj in RESTRICT_W.items():
        rows = _ys(r, dj)
        for di, wi in RESTRICT_W.items():
            out = out + (wj * wi) * np.roll(rows, -di, axis=1)
    return out[0::2, 0::2]


class Level:
    """Operator, diagonal and smoother parameters of one grid level."""

    def __init__(self, kind: str, n: int, c: float = 0.0, smoother="chebyshev",
                 degree=None, ratio=None, omega=None):
        self.kind, self.n, self.c = kind, n, c
        if kind == "ch":
            self.diag = ch_diagonal(n, c)
            lmax = ch_lmax(n, c)
            degree = 3 if degree is None else degree
            ratio = 16.0 if ratio is None else ratio
        elif kind == "lap":
            self.diag = lap_diagonal(n)
            lmax = LAP_LMAX
            degree = 2 if degree is None else degree
            ratio = 4.0 if ratio is None else ratio
        else:
            raise ValueError(kind)
        if smoother == "chebyshev":
            self.a, self.g = chebyshev_coefficients(lmax, ratio, degree)
        elif smoother == "jacobi":
            w = omega if omega is not None else (
                0.8 if kind == "lap" else 2 * (1 + 20 * c * float(n) ** 4)
                / (2 + 68 * c * float(n) ** 4))
            self.a, self.g = [w] * degree, [0.0] * degree
        else:
            raise ValueError(smoother)

    def apply(self, x):
        return apply_ch(x, self.c) if self.kind == "ch" else lap5(x)

    def coarse_solve(self, b):
        """Exact solve on the coarsest grid (dense; weighted-mean constraint
        for the Laplacian)."""
        if self.kind == "ch":
            A = dense.probe(self.apply, self.n)
            return np.linalg.solve(A, b.ravel()).reshape(b.shape)
        return dense.solve_poisson_dense(b, dense.probe(self.apply, self.n))


def hierarchy(kind: str, n: int, c: float = 0.0, **kw):
    levels = []
    while True:
        levels.append(Level(kind, n, c, **kw))
        if n <= COARSEST:
            break
        n //= 2
    return levels


def smooth(level: Level, x, b):
    """Polynomial smoother: x_{k+1} = x_k + a_k D^{-1}(b - A x_k) + g_k (x_k - x_{k-1})."""
    x_prev = x
    for a, g in zip(level.a, level.g):
        x_new = x + a * (b - level.apply(x)) / level.diag + g * (x - x_prev)
        x_prev, x = x, x_new
    return x


def vcycle(levels, b, depth=0):
    """z = V(b): one V-cycle from a zero initial guess, same smoother before
    and after the coarse correction (so the cycle is self-adjoint in W)."""
    lev = levels[depth]
    if depth == len(levels) - 1:
        return lev.coarse_solve(b)
    x = smooth(lev, np.zeros_like(b), b)
    r = b - lev.apply(x)
    e = vcycle(levels, restrict(r), depth + 1)
    x = x + prolong(e)
    return smooth(lev, x, b)


def project(x):
    return x - wmean(x)
