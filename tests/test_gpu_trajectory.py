"""Fifty time steps at 1024 x 1024 against the oracle's fifty steps (the
paper's scheme run as a trajectory, Sec. 4; u* held fixed): the phase field,
the pressure and the corrected velocity after step 1 and step 50 in float64
and with the float32 V-cycle, and the mass drift over the trajectory.

Bars: relative W-norm forward error of phi, p, u and v <= 1e-10 after one
step and after fifty (each step's solve stops at its tolerance or the float64
floor, and the step map is non-expansive on the stable modes, so the step
errors add up at most; measured on MI355X for phi: 7e-15 after one step,
4e-14 after fifty, in both precisions), mass drift <= 50 x 3e-14 relative
(the per-step bound of the three-step test; measured 1e-15).  The pressure
solve runs at PRESSURE_RTOL, the relative residual at which its forward error
meets the 1e-10 bar."""
import numpy as np
import pytest
import torch

import synthetic as S
import oracle.step
from oracle import ops

import paper_1811_11842_amd as bf  # loads the HIP library on first use; raises if it is missing

pytestmark = pytest.mark.gpu
PRM = S.DEFAULT_PARAMS
N, STEPS = 1024, 50
PRESSURE_RTOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def reference():
    phi0 = S.initial_phi(N)
    u0, v0 = S.inflow_velocity(N)
    traj = [phi0]
    flow = {}
    phi = phi0
    for k in range(1, STEPS + 1):
        phi, p, u, v = oracle.step.step(phi, u0, v0, **PRM)
        traj.append(phi)
        if k in (1, STEPS):
            flow[k] = (p, u, v)
    return u0, v0, traj, flow


def relw(a, b):
    return float(ops.wnorm(a - b) / ops.wnorm(b))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fifty_steps_match_oracle(dev, reference, prec):
    print(f"trajectory n={N} steps={STEPS} mg={prec}", flush=True)
    u0, v0, traj, flow = reference
    g = bf.Grid(N)
    mg = bf.MG_F32 if prec == "f32" else bf.MG_F64
    oc = bf.default_opts(bf.OP_CH, rtol=1e-10, mg_precision=mg)
    op = bf.default_opts(bf.OP_LAP, rtol=PRESSURE_RTOL, mg_precision=mg)
    phi = torch.from_numpy(traj[0].copy()).to(dev)
    us, vs = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
    p, u, v = g.field(), g.field(), g.field()
    errs, ferrs, iters = {}, {}, []
    for k in range(1, STEPS + 1):
        st = g.step(bf.make_params(**PRM), phi, us, vs, p, u, v, oc, op)
        assert st[0].status in (bf.OK, bf.AT_FLOOR) and st[1].status == bf.OK
        iters.append(st[0].iters)
        if k in (1, STEPS):
            torch.cuda.synchronize()
            errs[k] = relw(phi.cpu().numpy(), traj[k])
            ferrs[k] = [relw(t.cpu().numpy(), r) for t, r in zip((p, u, v), flow[k])]
    out = phi.cpu().numpy()
    dm = abs(float(ops.mass(out) - ops.mass(traj[0]))) / float(ops.mass(traj[0]))
    print(f"  error after 1 step {errs[1]:.2e}, after {STEPS} {errs[STEPS]:.2e}; "
          f"mass drift {dm:.1e}; CH iterations {iters[0]} .. {iters[-1]}; p, u, v errors "
          f"{ferrs[1][0]:.1e} {ferrs[1][1]:.1e} {ferrs[1][2]:.1e} (step 1), "
          f"{ferrs[STEPS][0]:.1e} {ferrs[STEPS][1]:.1e} {ferrs[STEPS][2]:.1e} (step {STEPS})")
    assert errs[1] <= 1e-10
    assert errs[STEPS] <= 1e-10
    assert max(ferrs[1]) <= 1e-10 and max(ferrs[STEPS]) <= 1e-10
    assert dm <= STEPS * 3e-14
