"""GPU parity of the variable-mobility Cahn-Hilliard step (the phi-dependent
mobility of eq. modCH, Sec. 2.2): the operator I + c L_m L (bf_apply_mob),
its GMRES solve (bf_solve_ch_mob) and the step (bf_step_ch_mob) against the
CPU oracle (oracle/mobility.py, long-double refined solves).

Tolerances: operator <= 1e-15 relative (double-double evaluation, one final
rounding, against long double); solves and steps <= 1e-10 relative W-norm
error (the float64 solve bar) at n = 64 and 256 (whole fields; the oracle's
sparse LU); at 1024 and 4096 the step is checked through properties that
hold at any size: the residual of the GPU result in the oracle's long-double
operator, b taken from the oracle, within max(2e-10, 4 floor_est) (rtol 1e-10
plus the rounding of b; at 4096^2 the float64 representation floor of this
operator, c n^4 m up to 8e6, lies above 1e-10 and the solve ends AT_FLOOR,
as the constant-mobility one does), and mass conservation; and at 4096^2
the variable-mobility path with a constant mobility field against the
long-double spectral solve of I + c M L^2 (forward error <= 1e-10)."""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle import mobility as mob
from oracle import ops

import paper_1811_11842_amd as bf  # loads the HIP library on first use; raises if it is missing

pytestmark = pytest.mark.gpu
PRM = S.DEFAULT_PARAMS
LD = np.longdouble


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


def D(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relw(a, b):
    return float(ops.wnorm(a - b) / ops.wnorm(b))


def gmres_opts(**kw):
    return bf.default_opts(bf.OP_CH, ksp=bf.KSP_GMRES, **kw)


@pytest.mark.parametrize("n", [64, 256])
def test_operator_matches_long_double_oracle(dev, n):
    print(f"apply_mob n={n}", flush=True)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n + 1, n))
    m = 0.02 + 0.3 * rng.random((n + 1, n))
    c = PRM["dt"] * PRM["kappa"]
    y = to_np(grid(n).apply_mob(c, D(m, dev), D(x, dev)))
    ref = mob.apply_mob(x.astype(LD), m.astype(LD), LD(c))
    e = relw(y.astype(LD), ref)
    print(f"  rel error {e:.2e}")
    assert e <= 1e-15


@pytest.mark.parametrize("n", [64, 256])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_solve_matches_oracle(dev, n, prec):
    print(f"solve_ch_mob n={n} {prec}", flush=True)
    phi = S.initial_phi(n)
    m = mob.mobility(phi, PRM["M"])
    b = mob.rhs_mob(phi, PRM["dt"], PRM["M"], PRM["Npoly"], PRM["chi"])
    c = PRM["dt"] * PRM["kappa"]
    ref = mob.solve(b, m, c)
    g = grid(n)
    x = g.field(0.0)
    st = g.solve_ch_mob(c, D(m, dev), D(b, dev), x,
                        gmres_opts(rtol=1e-12, mg_precision=bf.MG_F32 if prec == "f32" else bf.MG_F64))
    e = relw(to_np(x).astype(LD), ref)
    print(f"  status={st.status} iters={st.iters} res={st.rel_res_true:.2e} err={e:.2e}")
    assert st.status in (bf.OK, bf.AT_FLOOR)
    assert e <= 1e-10


def test_cg_is_rejected(dev):
    n = 64
    g = grid(n)
    with pytest.raises(bf.BiofilmError, match="GMRES"):
        g.solve_ch_mob(1e-7, g.field(0.1), g.field(0.3), g.field(0.0),
                       bf.default_opts(bf.OP_CH))


@pytest.mark.parametrize("n", [64, 256])
def test_step_matches_oracle(dev, n):
    print(f"step_ch_mob n={n}", flush=True)
    phi0 = S.initial_phi(n)
    ref = mob.step_mob(phi0, **{k: PRM[k] for k in ("dt", "M", "kappa", "Npoly", "chi",
                                                      "phi_lo", "phi_hi")})
    g = grid(n)
    phi = D(phi0, dev)
    st = g.step_ch_mob(bf.make_params(**PRM), phi, gmres_opts(rtol=1e-12))
    out = to_np(phi)
    e = relw(out.astype(LD), ref)
    dm = abs(float(ops.mass(out) - ops.mass(phi0))) / float(ops.mass(phi0))
    print(f"  status={st.status} iters={st.iters} err={e:.2e} mass drift {dm:.1e}")
    assert st.status in (bf.OK, bf.AT_FLOOR)
    assert e <= 1e-10
    assert dm <= 1e-13


def test_step_depends_only_on_its_arguments(dev):
    """bf_step_ch_mob keeps nothing between calls (its warm start is built from
    phi^n alone): a state stepped again after a step from another state gives
    bit-identical phi and iteration counts, and so does a fresh grid."""
    n = 256
    prm = bf.make_params(**PRM)
    o = gmres_opts(rtol=1e-12)
    g = grid(n)
    phi = D(S.initial_phi(n), dev)
    g.step_ch_mob(prm, phi, o)
    state = to_np(phi)  # one step in: the least-squares gamma is far from zero

    def one(grid_, ph):
        t = D(ph, dev)
        st = grid_.step_ch_mob(prm, t, o)
        return to_np(t), (st.iters, st.restarts)

    a, ia = one(g, state)
    one(g, S.initial_phi(n, seed=4242))
    b, ib = one(g, state)
    with bf.Grid(n) as h:
        c, ic = one(h, state)
    assert ia == ib == ic
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_uniform_state_is_a_fixed_point(dev):
    """A uniform phi has a constant mu and mobility: b = phi and the solution is
    phi.  (The preconditioned Krylov space is not the constant mode alone -- the
    smoother's diagonal differs next to the walls -- so the iterate is exact only
    to the solve's tolerance: rtol 1e-13, bound 1e-13 absolute.)"""
    n = 256
    g = grid(n)
    phi = g.field(0.25)
    st = g.step_ch_mob(bf.make_params(**PRM), phi, gmres_opts(rtol=1e-13))
    assert st.status in (bf.OK, bf.AT_FLOOR)
    assert np.abs(to_np(phi) - 0.25).max() <= 1e-13


@pytest.mark.parametrize("n", [1024, 4096])
def test_step_residual_and_mass_at_scale(dev, n):
    print(f"step_ch_mob n={n}", flush=True)
    phi0 = S.initial_phi(n)
    g = grid(n)
    phi = D(phi0, dev)
    o = gmres_opts(mg_precision=bf.MG_F32)
    st = g.step_ch_mob(bf.make_params(**PRM), phi, o)
    out = to_np(phi)
    print(f"  status={st.status} iters={st.iters} restarts={st.restarts} {st.ms:.1f} ms "
          f"res={st.rel_res_true:.2e} floor={st.floor_est:.1e}")
    assert st.status in (bf.OK, bf.AT_FLOOR)
    b = mob.rhs_mob(phi0, PRM["dt"], PRM["M"], PRM["Npoly"], PRM["chi"])
    m = mob.mobility(phi0, PRM["M"])
    r = b.astype(LD) - mob.apply_mob(out.astype(LD), m.astype(LD), LD(PRM["dt"] * PRM["kappa"]))
    rel = float(ops.wnorm(r) / ops.wnorm(b.astype(LD)))
    dm = abs(float(ops.mass(out) - ops.mass(phi0))) / float(ops.mass(phi0))
    print(f"  long-double residual {rel:.2e}  mass drift {dm:.1e}")
    assert rel <= max(2e-10, 4.0 * st.floor_est)
    assert dm <= 1e-13


def test_constant_mobility_field_at_4096_matches_spectral(dev):
    n, M = 4096, 0.3
    print(f"solve_ch_mob constant m n={n}", flush=True)
    from oracle import spectral
    phi0 = S.initial_phi(n)
    c = PRM["dt"] * PRM["kappa"]
    g = grid(n)
    x = g.field(0.0)
    st = g.solve_ch_mob(c, g.field(M), D(phi0, dev), x, gmres_opts(mg_precision=bf.MG_F32))
    ref = spectral.solve_ch(phi0.astype(LD), LD(c) * LD(M))
    e = relw(to_np(x).astype(LD), ref)
    print(f"  status={st.status} iters={st.iters} res={st.rel_res_true:.2e} "
          f"floor={st.floor_est:.1e} err={e:.2e}")
    assert st.status in (bf.OK, bf.AT_FLOOR)
    assert e <= 1e-10
