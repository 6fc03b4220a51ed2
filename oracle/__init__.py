"""CPU oracle for the biofilm-flow time step -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct numpy/scipy code that states what the GPU path
computes, written from the paper (McClanahan et al., "Parallel Simulations of
Biofilm Flow using the Modified Cahn-Hilliard Equation", arXiv:1811.11842):

  * ops       -- the 5-point Laplacian, the 13-point biharmonic, the
                 Cahn-Hilliard operator I + c*L^2, central divergence and
                 gradient, the trapezoid-weighted inner product (Sec. 4,
                 eq. discreteBC, Listing "Constructing the matrix with DMDA").
  * fh        -- Flory-Huggins energy density, its derivative mu_FH and the
                 right-hand side of the semi-implicit Cahn-Hilliard step
                 (Sec. 2.2 eq. modCH with the Flory-Huggins parameters of
                 the parameter table in Sec. 5).
  * spectral  -- exact solves by FFT(x) x DCT-I(y) diagonalisation, in float64
                 and in long double (the accuracy reference).
  * dense     -- dense assembly (two independent ways) and dense solves for
                 tiny grids.
  * cg        -- plain conjugate gradients in the weighted inner product.
  * mg        -- geometric-multigrid pieces and the V-cycle, written plainly.
  * step      -- one projection step (Sec. 4: eqs. pressuresolve and
                 velocityupdate) coupled with the Cahn-Hilliard solve.
  * cn        -- the Crank-Nicolson step with extrapolated chemical
                 potential (the paper's second-order time scheme, Sec. 4).
  * adjoint   -- the Cahn-Hilliard rollout with explicit advection (the flux
                 div(phi v) of eq. modCH) and its hand-derived adjoint: the
                 gradients of the upper-half mass with respect to chi, the
                 inflow speed and the initial phi.
  * momentum  -- the momentum predictor of the projection method (Sec. 4,
                 eq. nopressmomentum): explicit advection, theta-implicit
                 viscous term, i.e. one 5-point Helmholtz solve per velocity
                 component with Dirichlet walls.
  * mobility  -- the Cahn-Hilliard step with the phi-dependent mobility of
                 the modified equation (Sec. 2.2, eq. modCH): the
                 variable-coefficient operator I + dt*kappa*L_m L.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP path and must never be used as
a fallback for it.

Every function cites the passage it follows.  Pins (checks against what the
paper and mathematics fix, not against this code) live in tests/test_oracle_*.py.
"""
from . import ops, fh, spectral, dense, cg, mg, step, adjoint, cn, momentum, mobility  # noqa: F401
