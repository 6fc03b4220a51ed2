"""Cahn-Hilliard step with the phi-dependent mobility of the modified equation
(oracle; test infrastructure).

The paper's network transport (Sec. 2.2, eq. modCH) has the flux
lambda*phi*grad(delta f / delta phi): the mobility is proportional to the
network volume fraction.  With the chemical potential split as in the
constant-mobility step (Flory-Huggins part explicit, gradient-energy part
-kappa*Delta(phi) implicit) and the mobility frozen at the old state,
m = M*clamp(phi^n), one step is

    (I + dt*kappa*L_m L) phi^{n+1} = phi^n + dt*L_m mu_FH(clamp(phi^n)),

L_m f = div_h(m grad_h f): the conservative 5-point form with face
mobilities m_{i+1/2,j} = (m_ij + m_{i+1,j})/2, periodic in x and with the
even reflection of eq. discreteBC in y (for f and m alike).  L is the
5-point Laplacian of ops.  L_m is self-adjoint in the trapezoid inner
product and sums to zero against it, so the step conserves mass; the product
L_m L is not self-adjoint, so the solve needs a nonsymmetric method.

The exact solution of the linear system is computed by iterative refinement
whose residuals are evaluated in long double, each correction from a direct
sparse LU of the assembled matrix (n <= 512) or from GMRES preconditioned
with the constant-mobility spectral solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fh, ops, spectral

_DIRS = ((0, -1), (0, 1), (-1, 0), (1, 0))


def lap_mob(f: np.ndarray, m: np.ndarray) -> np.ndarray:
    """L_m f = (1/h^2) sum over the four faces of m_face (f_nb - f), m_face the
    mean of the two node mobilities; ghosts by reflection, columns wrap."""
    n = ops.n_of(f)
    h = f.dtype.type(1) / n
    acc = np.zeros_like(f)
    for dj, di in _DIRS:
        mf = (m + ops.shift(m, dj, di)) / 2
        acc = acc + mf * (ops.shift(f, dj, di) - f)
    return acc / (h * h)


def apply_mob(x: np.ndarray, m: np.ndarray, c) -> np.ndarray:
    """A_m x = x + c L_m L x."""
    return x + x.dtype.type(c) * lap_mob(ops.lap5(x), m)


def mobility(phi, M, lo=1e-6, hi=1.0 - 1e-6):
    """m = M * clamp(phi): the network-fraction proportional mobility."""
    return M * fh.clamp(phi, lo, hi)


def rhs_mob(phi, dt, M, Npoly, chi, lo=1e-6, hi=1.0 - 1e-6):
    """b = phi + dt L_m mu_FH(clamp(phi)), m = M clamp(phi)."""
    p = fh.clamp(phi, lo, hi)
    return phi + dt * lap_mob(fh.mu_fh(p, Npoly, chi), M * p)


def assemble(n: int, m: np.ndarray, c) -> sp.csr_matrix:
    """Sparse matrix of A_m = I + c L_m L (L_m and L by probing the stencil
    functions column by column is too slow beyond tiny grids, so both are
    built from their node coefficients: L_m row (i, j) has m_face n^2 at each
    neighbour and -sum m_face n^2 on the diagonal, reflected neighbours folded
    onto their mirror rows)."""
    size = (n + 1) * n
    n2 = float(n) * n

    def refl(j):
        j = -j if j < 0 else j
        return 2 * n - j if j > n else j

    def build(coef):
        rows, cols, vals = [], [], []
        for j in range(n + 1):
            for i in range(n):
                k = j * n + i
                diag = 0.0
                for dj, di in _DIRS:
                    jj, ii = refl(j + dj), (i + di) % n
                    w = coef(j, i, jj, ii)
                    rows.append(k); cols.append(jj * n + ii); vals.append(w * n2)
                    diag -= w * n2
                rows.append(k); cols.append(k); vals.append(diag)
        return sp.csr_matrix((vals, (rows, cols)), shape=(size, size))

    L = build(lambda j, i, jj, ii: 1.0)
    Lm = build(lambda j, i, jj, ii: (m[j, i] + m[jj, ii]) / 2)
    return (sp.identity(size, format="csr") + c * (Lm @ L)).tocsr()


def solve_direct(b: np.ndarray, m: np.ndarray, c) -> np.ndarray:
    """x = A_m^{-1} b by sparse LU (small grids)."""
    n = ops.n_of(b)
    return spla.spsolve(assemble(n, m, c).tocsc(), b.ravel()).reshape(b.shape)


def solve(b: np.ndarray, m: np.ndarray, c, tol=1e-17, max_refine=6) -> np.ndarray:
    """x = A_m^{-1} b by iterative refinement: residuals b - A_m x in long
    double, each correction from a float64 solve -- the sparse LU of the
    assembled matrix for n <= 512, else GMRES right-preconditioned by the
    exact solve of the constant-mobility operator I + c*mean_W(m)*L^2.
    Returns the long-double iterate once ||r||_W <= tol ||b||_W (or after
    max_refine corrections)."""
    n = ops.n_of(b)
    shape = b.shape
    L = np.longdouble
    bl = b.astype(L)
    ml = m.astype(L)
    x = np.zeros_like(bl)
    m64 = np.asarray(m, dtype=np.float64)
    if n <= 512:
        lu = spla.splu(assemble(n, m64, float(c)).tocsc())

        def correction(r64):
            return lu.solve(r64.ravel()).reshape(shape)
    else:
        cm = float(c) * float(ops.wmean(m64))
        A = spla.LinearOperator((b.size, b.size), dtype=np.float64,
                                matvec=lambda v: apply_mob(v.reshape(shape), m64, c).ravel())
        P = spla.LinearOperator((b.size, b.size), dtype=np.float64,
                                matvec=lambda v: spectral.solve_ch(v.reshape(shape), cm).ravel())

        def correction(r64):
            d, _ = spla.gmres(A, r64.ravel(), M=P, rtol=1e-13, atol=0.0, restart=60,
                              maxiter=50)
            return d.reshape(shape)
    bn = ops.wnorm(bl)
    if bn == 0:
        return x
    for _ in range(max_refine):
        r = bl - apply_mob(x, ml, L(c))
        if ops.wnorm(r) <= tol * bn:
            break
        x = x + correction(r.astype(np.float64)).astype(L)
    return x


def step_mob(phi, dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6, phi_lo=1e-6,
             phi_hi=1.0 - 1e-6, direct=False):
    """One step with the mobility M*clamp(phi^n) (long-double result unless direct)."""
    m = mobility(phi, M, phi_lo, phi_hi)
    b = rhs_mob(phi, dt, M, Npoly, chi, phi_lo, phi_hi)
    c = dt * kappa
    return solve_direct(b, m, c) if direct else solve(b, m, c)
