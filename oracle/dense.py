"""Dense matrices of the grid operators for tiny grids (oracle; test
infrastructure).

Two independent assemblies:
  * by probing: column e of the matrix is the operator applied to unit
    vector e (uses the stencil functions of ops);
  * explicitly, row by row, from the matrix row of Sec. 4.1 (Listing
    "Constructing the matrix with DMDA": 4 on the diagonal, -1 for the four
    neighbours, i.e. the matrix -h^2 L), with periodic column wrap (an index
    i-1 = -1 maps to the last column, Sec. 4.1) and ghost rows folded back onto
    interior rows by eq. discreteBC.  The biharmonic is then the matrix
    product L @ L, which shares nothing with the 13-point stencil code.

Unknown ordering: k = j*N + i (row-major, x fastest), matching the arrays.
"""
from __future__ import annotations

import numpy as np


def probe(op, n: int, dtype=np.float64) -> np.ndarray:
    """Matrix of a linear map on (N+1, N) fields, by unit-vector probing."""
    size = (n + 1) * n
    A = np.zeros((size, size), dtype=dtype)
    for k in range(size):
        e = np.zeros(size, dtype=dtype)
        e[k] = 1
        A[:, k] = op(e.reshape(n + 1, n)).ravel()
    return A


def lap_explicit(n: int, dtype=np.float64) -> np.ndarray:
    """Matrix of L from the paper's row values and boundary rules."""
    size = (n + 1) * n
    h2inv = dtype(n) * n
    A = np.zeros((size, size), dtype=dtype)
    row_vals = {(0, 0): 4.0, (-1, 0): -1.0, (1, 0): -1.0, (0, -1): -1.0, (0, 1): -1.0}
    for j in range(n + 1):
        for i in range(n):
            r = j * n + i
            for (di, dj), v in row_vals.items():
                ii = (i + di) % n            # periodic wrap, Sec. 4.1
                jj = j + dj
                if jj < 0:                   # phi[-1] = phi[1]
                    jj = -jj
                if jj > n:                   # phi[N+1] = phi[N-1]
                    jj = 2 * n - jj
                A[r, jj * n + ii] += -v * h2inv   # L = -(1/h^2) * (paper matrix)
    return A


def weight_vector(n: int, dtype=np.float64) -> np.ndarray:
    w = np.ones((n + 1, n), dtype=dtype)
    w[0, :] = 0.5
    w[-1, :] = 0.5
    return w.ravel()


def solve_ch_dense(b: np.ndarray, c, L: np.ndarray | None = None) -> np.ndarray:
    """x = (I + c L L)^{-1} b with the explicitly assembled L."""
    n = b.shape[1]
    if L is None:
        L = lap_explicit(n, b.dtype.type)
    A = np.eye(L.shape[0], dtype=L.dtype) + c * (L @ L)
    return np.linalg.solve(A, b.ravel()).reshape(b.shape)


def solve_poisson_dense(rhs: np.ndarray, L: np.ndarray | None = None) -> np.ndarray:
    """Bordered system [[L, 1], [w^T, 0]] [p; s] = [rhs - wmean(rhs); 0].

    The constraint w^T p = 0 fixes the constant of the singular Neumann
    problem (Sec. 4.1, null-space removal); the border column of ones is the
    right null vector of L.
    """
    n = rhs.shape[1]
    if L is None:
        L = lap_explicit(n, rhs.dtype.type)
    w = weight_vector(n, rhs.dtype.type)
    size = L.shape[0]
    B = np.zeros((size + 1, size + 1), dtype=L.dtype)
    B[:size, :size] = L
    B[:size, size] = 1
    B[size, :size] = w
    f = rhs.ravel() - (w @ rhs.ravel()) / w.sum()
    sol = np.linalg.solve(B, np.concatenate([f, [0.0]]))
    return sol[:size].reshape(rhs.shape)
