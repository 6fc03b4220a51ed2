"""Exact solves of the constant-coefficient grid operators (oracle; test
infrastructure).

With periodic x and the even reflection of eq. discreteBC in y, the 5-point
Laplacian L is diagonalised by Fourier modes in x times cosine modes in y:
    L [cos(2 pi k i / N) cos(pi l j / N)] = lam(k, l) * [same],
    lam(k, l) = -(4/h^2) (sin^2(pi k / N) + sin^2(pi l / (2N))),
k = 0..N-1, l = 0..N (the textbook fast Poisson solver idea).  The cosine
transform in y is the DCT of type I over the N+1 rows; the Cahn-Hilliard
operator I + c L^2 has eigenvalues 1 + c lam^2.

So the solutions of the linear systems A x = b of Sec. 4 (the Cahn-Hilliard
step and the Neumann pressure Poisson problem eq. pressuresolve) are computed
exactly (up to rounding) by transform -> divide -> inverse transform.  The
functions run in float64 or, for the accuracy reference, in long double.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .ops import n_of, wmean

PI_LD = np.longdouble("3.14159265358979323846264338327950288")


def _pi(dtype):
    return PI_LD.astype(dtype) if dtype == np.longdouble else np.float64(np.pi)


def lap_eigenvalues(n: int, dtype=np.float64) -> np.ndarray:
    """lam(k, l) for the rfft half-spectrum k = 0..N/2 and l = 0..N, shape (N+1, N/2+1)."""
    dtype = np.dtype(dtype).type
    pi = _pi(dtype)
    k = np.arange(n // 2 + 1, dtype=dtype)
    l = np.arange(n + 1, dtype=dtype)
    sx = np.sin(pi * k / n) ** 2
    sy = np.sin(pi * l / (2 * n)) ** 2
    return -(4 * dtype(n) * n) * (sx[None, :] + sy[:, None])


def lap_eigenvalue_full(n: int, k: int, l: int, dtype=np.float64):
    dtype = np.dtype(dtype).type
    pi = _pi(dtype)
    return -(4 * dtype(n) * n) * (np.sin(pi * dtype(k) / n) ** 2
                                  + np.sin(pi * dtype(l) / (2 * n)) ** 2)


def _forward(x):
    return sfft.rfft(sfft.dct(x, type=1, axis=0), axis=1)


def _inverse(xh, n):
    return sfft.idct(sfft.irfft(xh, n=n, axis=1), type=1, axis=0)


def solve_ch(b: np.ndarray, c) -> np.ndarray:
    """x = (I + c L^2)^{-1} b, exact up to rounding in b's dtype."""
    n = n_of(b)
    lam = lap_eigenvalues(n, b.dtype)
    c = b.dtype.type(c)
    return _inverse(_forward(b) / (1 + c * lam * lam), n)


def apply_ch_spectral(x: np.ndarray, c) -> np.ndarray:
    """A_CH x through the spectrum (used to evaluate residuals in long double
    independently of the stencil code)."""
    n = n_of(x)
    lam = lap_eigenvalues(n, x.dtype)
    c = x.dtype.type(c)
    return _inverse(_forward(x) * (1 + c * lam * lam), n)


def solve_poisson(rhs: np.ndarray) -> np.ndarray:
    """p with L p = rhs - wmean(rhs) and wmean(p) = 0.

    The all-Neumann problem is singular (Sec. 4.1: the null space of constants
    is removed from the right-hand side, Listing "Removing a nullspace").
    With the reflection the left null vector is the weight vector, so the
    compatible right-hand side has zero weighted mean; the (0,0) cosine/Fourier
    coefficient is proportional to the weighted sum and is set to zero in both
    the right-hand side and the solution.
    """
    n = n_of(rhs)
    lam = lap_eigenvalues(n, rhs.dtype)
    rh = _forward(rhs - wmean(rhs))
    lam = lam.copy()
    lam[0, 0] = 1
    ph = rh / lam
    ph[0, 0] = 0
    p = _inverse(ph, n)
    return p - wmean(p)
