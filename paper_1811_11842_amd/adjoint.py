"""Gradients of a Cahn-Hilliard rollout through the library's adjoint step.

A rollout maps (phi0, chi, U) to phi_N: N calls of bf_step_ch, each advected
by the projected inflow velocity (u, v) = P(U * base + noise_u, noise_v),
where P is the projection step of the paper (Sec. 4, eqs. pressuresolve and
velocityupdate: bf_pressure_rhs, bf_solve_pressure, bf_velocity_correct).
P is linear, so d(u, v)/dU = P(base, 0).

The reverse pass calls bf_adjoint_step once per step, last step first.  Only
every k-th state (a checkpoint) is kept in the forward pass; the states of a
segment are recomputed from its checkpoint just before the segment is
reversed, so memory is (N/k + k) fields instead of N.

`RolloutFn` wraps this as a torch.autograd.Function; `Rollout` holds the
fixed data (grid, step count, velocity profile and noise, solver options).
All arithmetic on fields runs in the library; this module sequences calls.
"""
from __future__ import annotations

import torch

from . import (NOT_CONVERGED, OP_CH, OP_LAP, MG_F64, Grid, SolverOpts, default_opts,
               make_params)


class ConvergenceError(RuntimeError):
    """A solve of the rollout (forward step, adjoint step or velocity
    projection) stopped at its iteration limit: the gradient would be built
    on an unconverged state, so none is returned."""


def _converged(st, what):
    if st.status == NOT_CONVERGED:
        raise ConvergenceError(f"{what}: not converged after {st.iters} iterations "
                               f"(relative residual {st.rel_res_true:.3e})")
    return st


class Rollout:
    """Fixed data of a differentiable rollout on one grid.

    base, noise_u, noise_v: device fields (u* = U * base + noise_u, v* = noise_v).
    params: dt, M, kappa, Npoly, phi_lo, phi_hi (chi is an input of the rollout).
    """

    def __init__(self, grid: Grid, steps: int, base, noise_u, noise_v, checkpoint_every=5,
                 rtol_forward=1e-12, rtol_adjoint=1e-12, rtol_pressure=1e-12,
                 mg_precision=MG_F64, **params):
        if steps < 1 or checkpoint_every < 1:
            raise ValueError("steps and checkpoint_every must be >= 1")
        self.g = grid
        self.steps = steps
        self.k = checkpoint_every
        self.base, self.noise_u, self.noise_v = base, noise_u, noise_v
        self.params = dict(params)
        self.opts_ch = default_opts(OP_CH, rtol=rtol_forward, mg_precision=mg_precision)
        self.opts_adj = default_opts(OP_CH, rtol=rtol_adjoint, mg_precision=mg_precision)
        self.opts_p = default_opts(OP_LAP, rtol=rtol_pressure, mg_precision=mg_precision)
        self.stats = []

    def _prm(self, chi):
        return make_params(chi=float(chi), **self.params)

    def _project(self, ustar, vstar):
        g, dt = self.g, self.params.get("dt", 1e-4)
        rhs = g.pressure_rhs(dt, ustar, vstar)
        p = g.field(0.0)
        _converged(g.solve_pressure(rhs, p, self.opts_p), "pressure solve")
        return g.velocity_correct(dt, p, ustar, vstar)

    def velocity(self, U):
        """(u, v, du, dv): projected velocity for inflow speed U and d/dU."""
        u, v = self._project(float(U) * self.base + self.noise_u, self.noise_v)
        du, dv = self._project(self.base.clone(), torch.zeros_like(self.base))
        return u, v, du, dv

    def forward(self, phi0, chi, U):
        """phi_N and the checkpoints {step index: state}."""
        prm = self._prm(chi)
        u, v, _, _ = self.velocity(U)
        phi = phi0.detach().clone()
        ckpt = {}
        for s in range(self.steps):
            if s % self.k == 0:
                ckpt[s] = phi.clone()
            self.stats.append(_converged(self.g.step_ch(prm, phi, u, v, self.opts_ch),
                                         f"forward step {s}"))
        return phi, ckpt

    def backward(self, lam_N, ckpt, chi, U):
        """(dJ/dphi0, dJ/dchi, dJ/dU) for lam_N = dJ/dphi_N."""
        prm = self._prm(chi)
        u, v, du, dv = self.velocity(U)
        lam = lam_N.detach().clone()
        gchi = gU = 0.0
        starts = sorted(ckpt)
        for s0 in reversed(starts):
            s1 = min(s0 + self.k, self.steps)
            states = [ckpt[s0].clone()]
            for _ in range(s0, s1 - 1):          # recompute the segment
                nxt = states[-1].clone()
                _converged(self.g.step_ch(prm, nxt, u, v, self.opts_ch), "recomputed step")
                states.append(nxt)
            for s in range(s1 - 1, s0 - 1, -1):
                lam, (a, b), st = self.g.adjoint_step(prm, states[s - s0], lam, lam, u, v,
                                                      du, dv, self.opts_adj)
                self.stats.append(_converged(st, f"adjoint step {s}"))
                gchi += a
                gU += b
        return lam, gchi, gU


class RolloutFn(torch.autograd.Function):
    """phi_N = RolloutFn.apply(phi0, chi, U, rollout); chi and U are 0-d
    float64 tensors (on any device)."""

    @staticmethod
    def forward(ctx, phi0, chi, U, rollout: Rollout):
        phiN, ckpt = rollout.forward(phi0, chi.item(), U.item())
        ctx.rollout = rollout
        ctx.ckpt = ckpt
        ctx.chi, ctx.U = chi.item(), U.item()
        ctx.dev = (chi.device, U.device)
        return phiN

    @staticmethod
    def backward(ctx, grad_phiN):
        lam, gchi, gU = ctx.rollout.backward(grad_phiN.contiguous(), ctx.ckpt, ctx.chi, ctx.U)
        return (lam, torch.tensor(gchi, dtype=torch.float64, device=ctx.dev[0]),
                torch.tensor(gU, dtype=torch.float64, device=ctx.dev[1]), None)


def upper_half_weights(grid: Grid):
    """h^2 W_j m_j with m = 1 above the middle row, 1/2 on it, 0 below: the
    trapezoid-rule weights of the integral of phi over y >= 1/2 (n even)."""
    n = grid.n
    w = torch.zeros(n + 1, 1, dtype=torch.float64, device=grid.device)
    w[n // 2 + 1:] = 1.0
    w[n // 2] = 0.5
    w[n] = 0.5
    return (w / (n * n)).expand(n + 1, n).contiguous()
