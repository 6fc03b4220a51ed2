"""Plain preconditioned conjugate gradients in the weighted inner product
(oracle; test infrastructure).

The paper solves its systems with a Krylov method and a Jacobi
preconditioner (Sec. 4.1, Listing "Creating PETSc KSP and PC objects").  The
operators with the even reflection of eq. discreteBC are self-adjoint and
positive definite (the Cahn-Hilliard operator) or semidefinite (minus the
Laplacian) in <x,y>_W, so CG in that inner product applies.  This is the
textbook algorithm with no fusion or reordering; it cross-checks the spectral
solver and is the iterative reference where no closed form exists.
"""
from __future__ import annotations

import numpy as np

from .ops import wdot, wnorm, wmean


def pcg(apply_a, b, x0=None, precond=None, rtol=1e-12, maxit=10000,
        project=False):
    """Solve A x = b; returns (x, iterations, relative W-residual history).

    precond(r) returns z ~ A^{-1} r (identity if None).  project=True removes
    the weighted mean from b, from every residual and from the result (the
    constant null space of the Neumann Laplacian).
    """
    b = b.copy()
    if project:
        b -= wmean(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = wnorm(b)
    if bn == 0:
        return np.zeros_like(b), 0, [0.0]
    r = b - apply_a(x)
    if project:
        r -= wmean(r)
    hist = [float(wnorm(r) / bn)]
    z = r if precond is None else precond(r)
    p = z.copy()
    rz = wdot(r, z)
    it = 0
    while hist[-1] > rtol and it < maxit:
        q = apply_a(p)
        alpha = rz / wdot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        if project:
            r -= wmean(r)
        it += 1
        hist.append(float(wnorm(r) / bn))
        if hist[-1] <= rtol:
            break
        z = r if precond is None else precond(r)
        rz_new = wdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    if project:
        x -= wmean(x)
    return x, it, hist


def jacobi_preconditioner(diag):
    """z = D^{-1} r with the operator's diagonal D (an array of the field shape)."""
    return lambda r: r / diag
