"""The allocation-free entry point bf_residual_noalloc, through the C ABI,
against the existing entry point bf_residual (accurate) on the same inputs:
r = b - A x must be bit-identical (the same double-double kernel) and the
device norms must equal bf_residual's host norms to a few ulps (the same
reductions in the same order; only the final square root and division run
on the device instead of the host).  Two calls in a row, the second with a
smaller grid, for every operator; rejected sizes; and replays of a captured
HIP graph that holds the call, each checked against the eager result."""
import ctypes

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import fh

import paper_1811_11842_amd as bf  # loads the HIP library on first use; raises if it is missing

pytestmark = pytest.mark.gpu
PRM = S.DEFAULT_PARAMS
C_CH = PRM["dt"] * PRM["M"] * PRM["kappa"]
COEF = {bf.OP_LAP: 0.0, bf.OP_CH: C_CH, bf.OP_HELM: 0.05}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def inputs(n, dev, seed):
    phi = S.initial_phi(n, seed=seed)
    b = fh.rhs_ch(phi, PRM["dt"], PRM["M"], PRM["Npoly"], PRM["chi"])
    x = phi + 1e-3 * S.random_field(n, seed + 1)
    return torch.from_numpy(b).to(dev), torch.from_numpy(x).to(dev)


def reference(n, op, b, x):
    """bf_residual (accurate) on a grid of n: (r, rel_norm, floor_est)."""
    with bf.Grid(n) as g:
        r, rel, fl = g.residual(op, COEF[op], b, x)
        torch.cuda.synchronize()
        return r.clone(), rel, fl


def close(a, b, ulps=4):
    return abs(a - b) <= ulps * 2.0 ** -52 * max(abs(a), abs(b))


@pytest.mark.parametrize("op", [bf.OP_LAP, bf.OP_CH, bf.OP_HELM])
@pytest.mark.parametrize("sizes", [(1024, 64), (4096, 128)])
def test_noalloc_residual_matches_existing_entry_point(dev, op, sizes):
    print(f"residual_noalloc op={op} sizes={sizes}", flush=True)
    results = []
    for k, n in enumerate(sizes):          # two calls in a row, the second smaller
        b, x = inputs(n, dev, 100 + 10 * k)
        r = torch.full_like(b, 5.0)
        norms = torch.full((3,), -1.0, dtype=torch.float64, device=dev)
        bf.residual_noalloc(op, COEF[op], b, x, r, norms)
        torch.cuda.synchronize()
        results.append((n, b, x, r.clone(), norms.cpu().numpy().copy()))
    for n, b, x, r, norms in results:
        rr, rel, fl = reference(n, op, b, x)
        bn = float(torch.sqrt((torch.cat([b[:1] * 0.5 ** 0.5, b[1:-1], b[-1:] * 0.5 ** 0.5]) ** 2)
                              .sum()))
        print(f"  n={n}: rel {norms[0]:.6e} ({rel:.6e}) floor {norms[1]:.6e} ({fl:.6e}) "
              f"||b|| {norms[2]:.6e} ({bn:.6e})")
        assert torch.equal(r, rr)
        assert close(norms[0], rel) and close(norms[1], fl)
        assert abs(norms[2] - bn) <= 1e-12 * bn


def test_noalloc_rejects_sizes_beyond_its_maximum(dev):
    b = torch.zeros(5, 4, dtype=torch.float64, device=dev)
    norms = torch.zeros(3, dtype=torch.float64, device=dev)
    L = bf.lib()
    P = ctypes.c_void_p
    for n in (65536, 100, 2):
        code = L.bf_residual_noalloc(n, bf.OP_CH, C_CH, P(b.data_ptr()), P(b.data_ptr()),
                                     P(norms.data_ptr()), P(norms.data_ptr()), None)
        assert code == bf.EINVAL, n
        assert b"powers of two" in L.bf_last_error()
    # null output and an unknown operator
    r = torch.zeros_like(b)
    assert L.bf_residual_noalloc(4, bf.OP_CH, C_CH, P(b.data_ptr()), P(b.data_ptr()),
                                 P(r.data_ptr()), None, None) == bf.EINVAL
    assert L.bf_residual_noalloc(4, 7, C_CH, P(b.data_ptr()), P(b.data_ptr()),
                                 P(r.data_ptr()), P(norms.data_ptr()), None) == bf.EINVAL


def test_noalloc_residual_in_a_captured_graph(dev):
    """The call captured once in a HIP graph and replayed three times, with
    eager work (new right-hand sides) between the replays: every replay
    matches bf_residual on that replay's inputs."""
    n = 256
    b, x = inputs(n, dev, 300)
    r = torch.zeros_like(b)
    norms = torch.zeros(3, dtype=torch.float64, device=dev)
    bf.residual_noalloc(bf.OP_CH, C_CH, b, x, r, norms)      # first call on this device: eager
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        bf.residual_noalloc(bf.OP_CH, C_CH, b, x, r, norms, stream=side)
    torch.cuda.synchronize()
    for k in range(3):
        nb, nx = inputs(n, dev, 310 + 5 * k)
        b.copy_(nb)
        x.copy_(nx)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        rr, rel, fl = reference(n, bf.OP_CH, b, x)
        got = norms.cpu().numpy()
        print(f"  replay {k}: rel {got[0]:.6e} ({rel:.6e})")
        assert torch.equal(r, rr)
        assert close(got[0], rel) and close(got[1], fl)
