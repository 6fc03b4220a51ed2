"""Grid operators of the discretised biofilm model (oracle; test infrastructure).

Grid (Sec. 4, Numerical Methods): nodes (x_i, y_j) = (i*dx, j*dy) on the unit
square, dx = dy = h = 1/N.  x is periodic (Sec. 2.4 boundary conditions;
Sec. 4.1: an index i-1 = -1 maps to the last column), so columns i = 0..N-1 are
stored.  y has rows j = 0..N with the no-flux condition realised by the
two-layer even reflection of eq. discreteBC:
    phi[-1] = phi[1], phi[-2] = phi[2], phi[N+1] = phi[N-1], phi[N+2] = phi[N-2].
Arrays are (N+1, N), indexed [j, i].

The dtype of the input is kept, so every function runs in float64 or in long
double (np.longdouble).
"""
from __future__ import annotations

import numpy as np


def n_of(x: np.ndarray) -> int:
    rows, cols = x.shape
    if rows != cols + 1:
        raise ValueError(f"expected shape (N+1, N), got {x.shape}")
    return cols


def reflect_rows(n: int, offset: int) -> np.ndarray:
    """Row index j+offset mapped back into 0..N by even reflection.

    Follows eq. discreteBC: index -k -> k and N+k -> N-k (|offset| <= 2 used).
    """
    j = np.arange(n + 1) + offset
    j = np.where(j < 0, -j, j)
    j = np.where(j > n, 2 * n - j, j)
    return j


def shift(x: np.ndarray, dj: int, di: int) -> np.ndarray:
    """Value at node (i+di, j+dj): periodic in x, even reflection in y."""
    n = n_of(x)
    return np.roll(x[reflect_rows(n, dj), :], -di, axis=1)


def weights(n: int, dtype=np.float64) -> np.ndarray:
    """Trapezoid weights of the rows: 1/2 on the wall rows j=0 and j=N, else 1.

    The 5-point Laplacian with even reflection is self-adjoint in
    <x, y>_W = sum_ij w_j x_ij y_ij (not in the plain dot product); this is
    the inner product used for every norm, mean and mass.
    """
    w = np.ones(n + 1, dtype=dtype)
    w[0] = w[-1] = 0.5
    return w[:, None]


def wdot(x: np.ndarray, y: np.ndarray) -> np.floating:
    """<x, y>_W (trapezoid in y, uniform in x)."""
    return np.sum(weights(n_of(x), x.dtype) * x * y)


def wnorm(x: np.ndarray) -> np.floating:
    return np.sqrt(wdot(x, x))


def wmean(x: np.ndarray) -> np.floating:
    """Weighted mean sum_W x / sum_W 1; sum_W 1 = N*N."""
    n = n_of(x)
    return wdot(x, np.ones_like(x)) / (x.dtype.type(n) * n)


def mass(x: np.ndarray) -> np.floating:
    """Trapezoid/periodic quadrature of the field over the unit square, h^2 sum_W x."""
    n = n_of(x)
    h = x.dtype.type(1) / n
    return h * h * wdot(x, np.ones_like(x))


def lap5(x: np.ndarray) -> np.ndarray:
    """Discrete Laplacian L x.

    Interior row of the matrix -h^2 L is (4, -1, -1, -1, -1) at
    (i,j), (i-1,j), (i+1,j), (i,j-1), (i,j+1) (Sec. 4.1, Listing
    "Constructing the matrix with DMDA"); the sign of L follows the continuous
    Laplacian.  Ghost rows come from eq. discreteBC; columns wrap.
    """
    n = n_of(x)
    h = x.dtype.type(1) / n
    return (shift(x, 0, -1) + shift(x, 0, 1) + shift(x, -1, 0) + shift(x, 1, 0)
            - 4 * x) / (h * h)


def bih13(x: np.ndarray) -> np.ndarray:
    """13-point discrete biharmonic, written out directly (not as L(Lx)).

    The fourth-order Cahn-Hilliard term needs a larger stencil (Sec. 1) and
    two ghost layers (eq. discreteBC).  Weights / h^4: centre 20; the four
    axis neighbours at distance 1: -8; the four diagonal neighbours: 2; the
    four axis neighbours at distance 2: 1.  With the two-layer reflection this
    equals L applied twice; that identity is a test, not an assumption here.
    """
    n = n_of(x)
    h = x.dtype.type(1) / n
    s = shift
    acc = 20 * x
    acc = acc - 8 * (s(x, 0, -1) + s(x, 0, 1) + s(x, -1, 0) + s(x, 1, 0))
    acc = acc + 2 * (s(x, -1, -1) + s(x, -1, 1) + s(x, 1, -1) + s(x, 1, 1))
    acc = acc + (s(x, 0, -2) + s(x, 0, 2) + s(x, -2, 0) + s(x, 2, 0))
    return acc / (h * h * h * h)


def apply_ch(x: np.ndarray, c) -> np.ndarray:
    """Cahn-Hilliard step operator A_CH x = x + c * Delta_h^2 x, c = dt*M*kappa.

    Backward Euler on the fourth-order term of eq. modCH (constant mobility
    M, gradient-energy coefficient kappa): the implicit part of the
    semi-implicit step (I + dt*M*kappa*Delta^2) phi^{n+1} = rhs.
    """
    return x + x.dtype.type(c) * bih13(x)


def divergence(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Central (2h) discrete divergence du/dx + dv/dy (Sec. 4: central differences).

    u wraps in x.  The wall-normal velocity v is odd across the walls
    (v . n = 0 at y = 0, 1, Sec. 4): v[-1] = -v[1], v[N+1] = -v[N-1].
    """
    n = n_of(u)
    h = u.dtype.type(1) / n
    dudx = (np.roll(u, -1, axis=1) - np.roll(u, 1, axis=1)) / (2 * h)
    vp = np.empty_like(v)
    vm = np.empty_like(v)
    vp[:-1] = v[1:]
    vp[-1] = -v[-2]          # v[N+1] = -v[N-1]
    vm[1:] = v[:-1]
    vm[0] = -v[1]            # v[-1] = -v[1]
    dvdy = (vp - vm) / (2 * h)
    return dudx + dvdy


def gradient(p: np.ndarray):
    """Central (2h) gradient (dp/dx, dp/dy); p even across the walls (dp/dn = 0,
    eq. pressuresolve), so dp/dy vanishes on the wall rows."""
    n = n_of(p)
    h = p.dtype.type(1) / n
    gx = (np.roll(p, -1, axis=1) - np.roll(p, 1, axis=1)) / (2 * h)
    gy = (shift(p, 1, 0) - shift(p, -1, 0)) / (2 * h)
    return gx, gy
