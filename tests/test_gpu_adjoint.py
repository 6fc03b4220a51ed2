"""GPU parity of the adjoint path (bf_step_ch with advection, bf_adjoint_step,
and the checkpointed rollout gradient) against the CPU oracle, and of the
rollout gradient against central finite differences of the GPU forward
rollout.

Tolerances
  * one advected step: relative W-norm error <= 1e-10 (the float64 solve bar);
  * one adjoint step: lambda_out relative <= 1e-9 and the two scalar
    contributions relative <= 1e-8 (transpose solve at rtol 1e-12; the oracle
    solves exactly);
  * rollout gradients vs the oracle: relative <= 1e-8, at 64 x 64 (6 steps)
    and at the configured 2048 x 2048 (20 steps);
  * rollout gradients vs finite differences: relative <= 1e-6.  The finite
    differences carry the rounding of J divided by eps; J is about 1e-2 and
    accurate to about 4e-17 here, so the small scalars dJ/dchi and dJ/dU take
    eps = 1e-4 (truncation error below 1e-8 relative; the eps = 1e-6 value of
    dJ/dchi is printed beside it), the directional derivatives in phi0 (order
    1e-2) eps = 1e-6; dJ/dU (about 1e-11) is below what the difference
    quotient resolves and gets an absolute bound (see _fd_check).
"""
import os
import time

import numpy as np
import pytest
import scipy.fft
import torch

import synthetic as S
from oracle import adjoint as adj
from oracle import ops

import paper_1811_11842_amd as bf  # loads the HIP library on first use; raises if it is missing
from paper_1811_11842_amd import adjoint as bfa

pytestmark = pytest.mark.gpu
WORKERS = max(1, min(16, os.cpu_count() or 1))
PRM = dict(dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0)
CHI = 0.6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


_grids = {}


def grid(n):
    if n not in _grids:
        _grids[n] = bf.Grid(n)
    return _grids[n]


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relw(a, b):
    return float(ops.wnorm(a - b) / ops.wnorm(b))


def setup(n):
    phi0 = S.initial_phi(n)
    Y, _ = S.node_coords(n)
    base = Y * (2.0 - Y)
    nu, nv = S.inflow_velocity(n, U=0.0)
    return phi0, base, nu, nv


@pytest.mark.parametrize("n", [64, 256])
def test_advected_step_matches_oracle(dev, n):
    print(f"step_ch advected n={n}", flush=True)
    phi0, base, nu, nv = setup(n)
    u, v, _, _ = adj.velocity(n, 1.0, PRM["dt"], nu, nv, base)
    ref = adj.step_adv(phi0, u, v, chi=CHI, **PRM)
    g = grid(n)
    phi = to_dev(phi0, dev)
    st = g.step_ch(bf.make_params(chi=CHI, **PRM), phi, to_dev(u, dev), to_dev(v, dev),
                   bf.default_opts(bf.OP_CH, rtol=1e-12))
    assert st.status in (bf.OK, bf.AT_FLOOR)
    assert relw(to_np(phi), ref) <= 1e-10
    # without velocity it is the Cahn-Hilliard half of the plain step
    phi = to_dev(phi0, dev)
    g.step_ch(bf.make_params(chi=CHI, **PRM), phi, None, None,
              bf.default_opts(bf.OP_CH, rtol=1e-12))
    assert relw(to_np(phi), adj.step_adv(phi0, None, None, chi=CHI, **PRM)) <= 1e-10


@pytest.mark.parametrize("n", [64, 256])
def test_adjoint_step_matches_oracle(dev, n):
    print(f"adjoint_step n={n}", flush=True)
    phi0, base, nu, nv = setup(n)
    u, v, du, dv = adj.velocity(n, 1.0, PRM["dt"], nu, nv, base)
    lam = adj.objective_weights(n) + 1e-3 * S.random_field(n, 17) / (n * n)
    ref, rc, ru = adj.adjoint_step(phi0, u, v, du, dv, lam, chi=CHI, **PRM)
    g = grid(n)
    D = lambda a: to_dev(a, dev)  # noqa: E731
    out, (gc, gu), st = g.adjoint_step(bf.make_params(chi=CHI, **PRM), D(phi0), D(lam), None,
                                       D(u), D(v), D(du), D(dv),
                                       bf.default_opts(bf.OP_CH, rtol=1e-12))
    print(f"  status={st.status} iters={st.iters} gchi={gc:.6e} ({rc:.6e}) gU={gu:.6e} ({ru:.6e})")
    assert st.status in (bf.OK, bf.AT_FLOOR)
    assert relw(to_np(out), ref) <= 1e-9
    assert abs(gc - rc) <= 1e-8 * abs(rc)
    assert abs(gu - ru) <= 1e-8 * abs(ru) + 1e-18
    # in place (lambda_out aliasing lambda_in) gives the same result
    lam_d = D(lam)
    out2, (gc2, gu2), _ = g.adjoint_step(bf.make_params(chi=CHI, **PRM), D(phi0), lam_d, lam_d,
                                         D(u), D(v), D(du), D(dv),
                                         bf.default_opts(bf.OP_CH, rtol=1e-12))
    assert torch.equal(out2, out) and gc2 == gc and gu2 == gu


def _rollout(n, steps, k, dev):
    phi0, base, nu, nv = setup(n)
    ro = bfa.Rollout(grid(n), steps, to_dev(base, dev), to_dev(nu, dev), to_dev(nv, dev),
                     checkpoint_every=k, rtol_forward=1e-13, rtol_adjoint=1e-13,
                     rtol_pressure=1e-13, **PRM)
    return phi0, base, nu, nv, ro


def _grad(ro, phi0, chi, U, dev):
    p = to_dev(phi0, dev).requires_grad_(True)
    c = torch.tensor(chi, dtype=torch.float64, requires_grad=True)
    u = torch.tensor(U, dtype=torch.float64, requires_grad=True)
    w = bfa.upper_half_weights(ro.g)
    J = (w * bfa.RolloutFn.apply(p, c, u, ro)).sum()
    J.backward()
    return J.item(), to_np(p.grad), c.grad.item(), u.grad.item()


def _J(ro, phi0, chi, U, dev):
    with torch.no_grad():
        phiN, _ = ro.forward(to_dev(phi0, dev), chi, U)
        return (bfa.upper_half_weights(ro.g) * phiN).sum().item()


def test_rollout_gradient_matches_oracle(dev):
    n, steps, k = 64, 6, 2
    phi0, base, nu, nv, ro = _rollout(n, steps, k, dev)
    J, gphi, gchi, gU = _grad(ro, phi0, CHI, 1.0, dev)
    rJ, rphi, rchi, rU = adj.rollout_grad(phi0, 1.0, steps, nu, nv, base, chi=CHI, **PRM)
    print(f"J={J:.15e} ({rJ:.15e}) gchi={gchi:.6e} ({rchi:.6e}) gU={gU:.6e} ({rU:.6e})")
    assert abs(J - rJ) <= 1e-12 * abs(rJ)
    assert relw(gphi, rphi) <= 1e-8
    assert abs(gchi - rchi) <= 1e-8 * abs(rchi)
    assert abs(gU - rU) <= 1e-8 * abs(rU) + 1e-15


def _fd_check(n, steps, k, ndir, dev):
    phi0, base, nu, nv, ro = _rollout(n, steps, k, dev)
    t0 = time.perf_counter()
    J, gphi, gchi, gU = _grad(ro, phi0, CHI, 1.0, dev)
    t_grad = time.perf_counter() - t0
    e = 1e-4
    fd_chi = (_J(ro, phi0, CHI + e, 1.0, dev) - _J(ro, phi0, CHI - e, 1.0, dev)) / (2 * e)
    fd_U = (_J(ro, phi0, CHI, 1.0 + e, dev) - _J(ro, phi0, CHI, 1.0 - e, dev)) / (2 * e)
    e6 = 1e-6
    fd6_chi = (_J(ro, phi0, CHI + e6, 1.0, dev) - _J(ro, phi0, CHI - e6, 1.0, dev)) / (2 * e6)
    print(f"n={n} steps={steps}: J={J:.12e}  gradient pass {t_grad:.2f} s")
    print(f"  dJ/dchi adjoint {gchi:.10e}  fd(1e-4) {fd_chi:.10e}  fd(1e-6) {fd6_chi:.10e}  "
          f"rel {abs(gchi - fd_chi) / abs(fd_chi):.2e}")
    print(f"  dJ/dU   adjoint {gU:.10e}  fd(1e-4) {fd_U:.10e}  "
          f"rel {abs(gU - fd_U) / max(abs(fd_U), 1e-300):.2e}")
    assert abs(gchi - fd_chi) <= 1e-6 * abs(fd_chi)
    # dJ/dU is about 1e-11: the finite difference cannot resolve it to 1e-6
    # relative in float64.  J (about 1e-2) is evaluated to about 4e-17
    # (solves at the float64 floor, 4M-term sum), so the difference quotient
    # carries up to 4e-17 / eps = 4e-13 of noise; the bound is 1e-12 absolute.
    # (The U gradient is held to 1e-8 relative against the oracle, whose own
    # U gradient is pinned by finite differences on the CPU.)
    assert abs(gU - fd_U) <= 1e-6 * abs(fd_U) + 1e-12
    rng = np.random.default_rng(2024)
    worst = 0.0
    for _ in range(ndir):
        d = rng.standard_normal(phi0.shape)
        fd = (_J(ro, phi0 + e6 * d, CHI, 1.0, dev) - _J(ro, phi0 - e6 * d, CHI, 1.0, dev)) / (2 * e6)
        ad = float(np.sum(gphi * d))
        worst = max(worst, abs(ad - fd) / abs(fd))
    print(f"  dJ/dphi0 . d over {ndir} seeded directions: worst rel {worst:.2e}")
    assert worst <= 1e-6
    return phi0, base, nu, nv, (J, gphi, gchi, gU)


def test_rollout_gradient_matches_finite_differences_256(dev):
    _fd_check(256, 10, 5, 4, dev)


@pytest.mark.timeout(900)
def test_rollout_gradient_2048_20_steps(dev):
    """The differentiation configuration: 2048 x 2048, float64, 20 steps,
    checkpoints every 5 steps: dJ/dchi, dJ/dU and 16 seeded directions of
    dJ/dphi0 against central finite differences, and J, dJ/dchi, dJ/dU and
    the whole field dJ/dphi0 against the oracle's rollout gradient (all
    states kept, exact spectral solves) to 1e-8 relative, which pins dJ/dU
    (about 1e-11, below what the difference quotient resolves) at this size."""
    n, steps = 2048, 20
    phi0, base, nu, nv, (J, gphi, gchi, gU) = _fd_check(n, steps, 5, 16, dev)
    with scipy.fft.set_workers(WORKERS):
        rJ, rphi, rchi, rU = adj.rollout_grad(phi0, 1.0, steps, nu, nv, base, chi=CHI, **PRM)
    e_phi = relw(gphi, rphi)
    print(f"  vs oracle: J {abs(J - rJ) / abs(rJ):.1e}  dJ/dphi0 {e_phi:.1e}  "
          f"dJ/dchi {abs(gchi - rchi) / abs(rchi):.1e}  dJ/dU {abs(gU - rU) / abs(rU):.1e} "
          f"({gU:.10e} vs {rU:.10e})")
    assert abs(J - rJ) <= 1e-12 * abs(rJ)
    assert e_phi <= 1e-8
    assert abs(gchi - rchi) <= 1e-8 * abs(rchi)
    assert abs(gU - rU) <= 1e-8 * abs(rU)


def test_rollout_raises_when_a_solve_does_not_converge(dev):
    """A rollout whose forward solves stop at the iteration limit (maxit 1)
    raises instead of returning a gradient; so does one whose adjoint solves
    stop there."""
    n, steps = 64, 2
    phi0, base, nu, nv, ro = _rollout(n, steps, 1, dev)
    ro.opts_ch.maxit = 1
    with pytest.raises(bfa.ConvergenceError, match="forward step"):
        _grad(ro, phi0, CHI, 1.0, dev)
    phi0, base, nu, nv, ro = _rollout(n, steps, 1, dev)
    ro.opts_adj.maxit = 1
    with pytest.raises(bfa.ConvergenceError, match="adjoint step"):
        _grad(ro, phi0, CHI, 1.0, dev)
    phi0, base, nu, nv, ro = _rollout(n, steps, 1, dev)
    ro.opts_p.maxit = 1
    with pytest.raises(bfa.ConvergenceError, match="pressure solve"):
        _grad(ro, phi0, CHI, 1.0, dev)
