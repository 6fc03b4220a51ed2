"""The largest grid the library accepts: n = 32768 (32769 x 32768 nodes,
1.07e9 points, 8.6 GB per float64 field), checked through properties that
hold at any size, so that index arithmetic at full size is exercised.

Input: the discrete eigenmode x(j, i) = cos(pi l j / n) cos(2 pi k i / n) of
the reflected 5-point Laplacian (Sec. 4, eq. discreteBC), formed on the
device as the outer product of two 1-D vectors computed on the host; its
eigenvalue lambda_L(k, l) is the closed form of oracle/spectral.py, and the
13-point operator's is 1 + c lambda_L^2.  Distinct k and l make a transposed
or shifted index visible (it breaks the eigen relation by O(s |x|)).

  - bf_apply, 5-point and 13-point: max |y - lambda x| <= 8 u sum|w| max|x|
    (the per-entry rounding bound of the smaller-size operator tests);
  - bf_solve_pressure on that mode: the solution is x / lambda_L; since L is
    W-self-adjoint with smallest nonzero |eigenvalue| lambda_min, the
    relative W-norm error is at most (|lambda_L| / lambda_min) times the
    relative true residual, which the solve reports."""
import numpy as np
import pytest
import torch

from oracle import spectral

import paper_1811_11842_amd as bf  # loads the HIP library on first use; raises if it is missing

pytestmark = pytest.mark.gpu
N = 32768
K, L = 3, 5
U = 2.0 ** -53
C_CH = 1e-4 * 1e-3  # dt * kappa


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def setup(dev):
    print(f"max-size grid n={N}", flush=True)
    g = bf.Grid(N)
    a = np.cos(np.pi * L * np.arange(N + 1) / N)
    b = np.cos(2 * np.pi * K * np.arange(N) / N)
    x = torch.outer(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)).contiguous()
    w = torch.ones(N + 1, 1, dtype=torch.float64, device=dev)
    w[0] = w[-1] = 0.5
    yield g, x, w
    g.close()
    del x
    torch.cuda.empty_cache()


def wnorm(v, w):
    return float(torch.sqrt((w * v * v).sum()))


@pytest.mark.parametrize("op", ["lap", "ch"])
def test_apply_eigenmode_at_max_size(setup, op):
    g, x, _ = setup
    lam = float(spectral.lap_eigenvalue_full(N, K, L))
    if op == "lap":
        y = g.apply(bf.OP_LAP, 0.0, x)
        ev, wsum = lam, 8.0 * N * N
    else:
        y = g.apply(bf.OP_CH, C_CH, x)
        ev, wsum = 1.0 + C_CH * lam * lam, 1.0 + 64.0 * C_CH * float(N) ** 4
    err = float((y - ev * x).abs().max())
    print(f"  {op}: lambda {ev:.6e}, max error {err:.2e}, bound {8 * U * wsum:.2e}")
    assert err <= 8 * U * wsum
    del y


def test_pressure_solve_at_max_size(setup):
    g, x, w = setup
    lam = float(spectral.lap_eigenvalue_full(N, K, L))
    lam_min = abs(float(spectral.lap_eigenvalue_full(N, 0, 1)))
    p = torch.zeros_like(x)
    st = g.solve_pressure(x, p, bf.default_opts(bf.OP_LAP, rtol=1e-8))
    exact = x / lam
    fe = wnorm(p - exact, w) / wnorm(exact, w)
    bound = abs(lam) / lam_min * st.rel_res_true * 1.01
    print(f"  pressure: iters {st.iters} status {st.status} true residual "
          f"{st.rel_res_true:.2e} forward error {fe:.2e} (bound {bound:.2e})")
    assert st.status == bf.OK
    assert st.rel_res_true <= 1e-8
    assert fe <= bound
    del p, exact
