"""The benchmark's configuration as a trajectory: 4096 x 4096, twenty time
steps from the seeded initial state (Sec. 4: the semi-implicit Cahn-Hilliard
step of eq. modCH, then the projection of eqs. pressuresolve and
velocityupdate; u* held fixed), in float64 and with the float32 V-cycle,
against the oracle's twenty steps.

Bars, checked after steps 1, 2, 10 and 20:
  * phi, p, u, v: relative W-norm forward error <= 1e-10 against the oracle
    (each step's solve stops at its tolerance or at the float64 floor, and the
    step map does not amplify the stable modes, so step errors add at most);
  * every checked Cahn-Hilliard solve: the oracle-recomputed float64 residual
    of the GPU's phi^{k} for the right-hand side of the GPU's phi^{k-1} is
    <= max(rtol, 4 rho_fl), rho_fl the float64 residual of the oracle's own
    float64 spectral solution of the same system (the rounding floor of the
    operator at this size: about 1e-7 after the first step, where ||b|| is
    small and c/h^4 = 2.8e7);
  * mass drift over the trajectory <= 20 x 3e-14 relative.
The pressure right-hand side does not depend on phi and u* is fixed, so p,
u, v are the same system every step; the pressure solve runs at
PRESSURE_RTOL, the relative residual at which its forward error meets the
1e-10 bar at this size.
"""
import os

import numpy as np
import pytest
import scipy.fft
import torch

import oracle.step
import synthetic as S
from oracle import fh, ops, spectral

import paper_1811_11842_amd as bf  # loads the HIP library on first use; raises if it is missing

pytestmark = pytest.mark.gpu
PRM = S.DEFAULT_PARAMS
C_CH = PRM["dt"] * PRM["M"] * PRM["kappa"]
N, STEPS = 4096, 20
CHECKED = (1, 2, 10, 20)
RTOL = 1e-10
PRESSURE_RTOL = 1e-12
WORKERS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def reference():
    """The oracle's trajectory at the checked steps (and the initial state)."""
    phi0 = S.initial_phi(N)
    u0, v0 = S.inflow_velocity(N)
    keep = {0: phi0}
    phi = phi0
    with scipy.fft.set_workers(WORKERS):
        for k in range(1, STEPS + 1):
            phi, p, u, v = oracle.step.step(phi, u0, v0, **PRM)
            if k in CHECKED:
                keep[k] = (phi, p, u, v)
            print(f"oracle step {k}", flush=True)
    return u0, v0, keep


def relw(a, b):
    return float(ops.wnorm(a - b) / ops.wnorm(b))


def _residual_and_floor(phi_prev, phi_new):
    """(float64 relative residual of phi_new for the step from phi_prev, the
    float64 floor rho_fl of that system), both evaluated by the oracle."""
    b = fh.rhs_ch(phi_prev, PRM["dt"], PRM["M"], PRM["Npoly"], PRM["chi"],
                  PRM["phi_lo"], PRM["phi_hi"])
    nb = ops.wnorm(b)
    res = float(ops.wnorm(b - ops.apply_ch(phi_new, C_CH)) / nb)
    x = spectral.solve_ch(b, C_CH)
    rho = float(ops.wnorm(b - ops.apply_ch(x, C_CH)) / nb)
    return res, rho


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_benchmark_trajectory_matches_oracle(dev, reference, prec):
    print(f"trajectory n={N} steps={STEPS} mg={prec}", flush=True)
    u0, v0, ref = reference
    mg = bf.MG_F32 if prec == "f32" else bf.MG_F64
    oc = bf.default_opts(bf.OP_CH, rtol=RTOL, mg_precision=mg)
    op = bf.default_opts(bf.OP_LAP, rtol=PRESSURE_RTOL, mg_precision=mg)
    prm = bf.make_params(**PRM)
    with bf.Grid(N) as g:
        phi = torch.from_numpy(ref[0].copy()).to(dev)
        us, vs = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
        p, u, v = g.field(), g.field(), g.field()
        states = {0: ref[0]}
        fields = {}
        for k in range(1, STEPS + 1):
            sc, sp = g.step(prm, phi, us, vs, p, u, v, oc, op)
            print(f"  step {k}: CH {sc.iters} it {bf.STATUS_NAMES[sc.status]} "
                  f"res {sc.rel_res_true:.2e} floor {sc.floor_est:.2e} | "
                  f"P {sp.iters} it res {sp.rel_res_true:.2e}", flush=True)
            assert sc.status in (bf.OK, bf.AT_FLOOR) and sp.status == bf.OK
            if k in CHECKED or k + 1 in CHECKED:
                torch.cuda.synchronize()
                states[k] = phi.cpu().numpy()
            if k in CHECKED:
                fields[k] = tuple(t.cpu().numpy() for t in (p, u, v))
    with scipy.fft.set_workers(WORKERS):
        for k in CHECKED:
            rphi, rp, ru, rv = ref[k]
            gp, gu, gv = fields[k]
            e = [relw(states[k], rphi), relw(gp, rp), relw(gu, ru), relw(gv, rv)]
            res, rho = _residual_and_floor(states[k - 1], states[k])
            print(f"  after step {k}: errors phi {e[0]:.2e} p {e[1]:.2e} u {e[2]:.2e} "
                  f"v {e[3]:.2e}; CH residual {res:.2e} (4 rho_fl {4 * rho:.2e})", flush=True)
            assert max(e) <= 1e-10
            assert res <= max(RTOL, 4 * rho)
    m0 = float(ops.mass(ref[0]))
    dm = abs(float(ops.mass(states[STEPS])) - m0) / m0
    print(f"  mass drift over {STEPS} steps {dm:.1e}")
    assert dm <= STEPS * 3e-14
