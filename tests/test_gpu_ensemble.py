"""GPU parity of the batched ensemble (bf_ensemble_*): every instance of an
uneven ensemble against the CPU oracle step with that instance's parameters
(relative W-norm error <= 1e-10 for phi, p, u, v, the float64 bar of the
single grid; the pressure solves run at rtol 1e-12, where p meets it), against the single-grid path, and the edge cases
of the batch (an instance whose pressure right-hand side vanishes, so it is
masked from the first iteration, next to instances that iterate)."""
import os

import numpy as np
import pytest
import scipy.fft
import torch

import oracle
import synthetic as S
from oracle import ops

import paper_1811_11842_amd as bf  # loads the HIP library on first use; raises if it is missing

pytestmark = pytest.mark.gpu
WORKERS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def relw(a, b):
    return float(ops.wnorm(a - b) / ops.wnorm(b))


def pack(ens, arrays, dev):
    t = torch.zeros(ens.total, dtype=torch.float64)
    for i, a in enumerate(arrays):
        o = ens.offsets[i]
        t[o:o + a.size] = torch.from_numpy(np.ascontiguousarray(a).ravel())
    return t.to(dev)


def unpack(ens, t, i):
    torch.cuda.synchronize()
    return ens.view(t, i).cpu().numpy()


def run(specs, dev, steps=1, zero_flow=()):
    inst = [S.ensemble_instance(s) for s in specs]
    if zero_flow:
        inst = [(ph, np.zeros_like(u) if k in zero_flow else u,
                 np.zeros_like(v) if k in zero_flow else v, prm)
                for k, (ph, u, v, prm) in enumerate(inst)]
    ens = bf.Ensemble([s["n"] for s in specs])
    phi = pack(ens, [a[0] for a in inst], dev)
    us = pack(ens, [a[1] for a in inst], dev)
    vs = pack(ens, [a[2] for a in inst], dev)
    p, u, v = ens.field(0.0), ens.field(0.0), ens.field(0.0)
    prms = [bf.make_params(**a[3]) for a in inst]
    stats = []
    for _ in range(steps):
        st, ms = ens.step(prms, phi, us, vs, p, u, v, bf.default_opts(bf.OP_CH, rtol=1e-10),
                          bf.default_opts(bf.OP_LAP, rtol=1e-12))
        stats.append(st)
    return ens, inst, phi, p, u, v, stats, ms


def test_layout_and_classes(dev):
    ens = bf.Ensemble([256, 128, 256, 512, 128])
    # classes by size, instances in input order within a class, blocks contiguous
    assert ens.info()[0][:2] == (128, 2) and ens.info()[1][:2] == (256, 2)
    assert ens.info()[2][:2] == (512, 1)
    assert all(r in (4, 5, 8) for _, _, r in ens.info())  # the autotuner's tile heights
    o = ens.offsets
    assert o[1] == 0 and o[4] == 129 * 128 and o[0] == 2 * 129 * 128
    assert o[2] == o[0] + 257 * 256 and o[3] == o[2] + 257 * 256
    assert ens.total == o[3] + 513 * 512
    with pytest.raises(bf.BiofilmError, match="EINVAL"):
        bf.Ensemble([64])
    with pytest.raises(bf.BiofilmError, match="EINVAL"):
        bf.Ensemble([300])


def test_ensemble_step_matches_oracle(dev):
    specs = S.ensemble_specs(7, seed=11, sizes=(128, 256, 512))
    ens, inst, phi, p, u, v, stats, ms = run(specs, dev)
    print("classes", ens.info(), f"step {ms:.1f} ms")
    for i, (ph0, u0, v0, prm) in enumerate(inst):
        rphi, rp, ru, rv = oracle.step.step(ph0, u0, v0, **prm)
        e = (relw(unpack(ens, phi, i), rphi), relw(unpack(ens, p, i), rp),
             relw(unpack(ens, u, i), ru), relw(unpack(ens, v, i), rv))
        sc, sp = stats[0][i]
        print(f"  inst {i} n={specs[i]['n']} chi={specs[i]['chi']:.3f} dt={specs[i]['dt']:.2e}: "
              f"CH it={sc.iters} {bf.STATUS_NAMES[sc.status]}  P it={sp.iters}  err {e}")
        assert sc.status in (bf.OK, bf.AT_FLOOR) and sp.status == bf.OK
        assert e[0] <= 1e-10 and e[1] <= 1e-10 and e[2] <= 1e-10 and e[3] <= 1e-10


def test_single_instance_class_matches_oracle(dev):
    """A size class holding one instance (a batch of one) takes its
    coefficients from the per-instance records like larger classes."""
    specs = S.ensemble_specs(3, seed=21, sizes=(128,))
    specs[2]["n"] = 256
    ens, inst, phi, p, u, v, stats, _ = run(specs, dev)
    assert sorted(c[:2] for c in ens.info()) == [(128, 2), (256, 1)]
    for i, (ph0, u0, v0, prm) in enumerate(inst):
        rphi, rp, ru, rv = oracle.step.step(ph0, u0, v0, **prm)
        sc, sp = stats[0][i]
        assert sc.status in (bf.OK, bf.AT_FLOOR) and sp.status == bf.OK
        assert relw(unpack(ens, phi, i), rphi) <= 1e-10
        assert relw(unpack(ens, p, i), rp) <= 1e-10


def test_ensemble_agrees_with_single_grid(dev):
    specs = S.ensemble_specs(4, seed=5, sizes=(128, 256))
    ens, inst, phi, p, u, v, stats, _ = run(specs, dev)
    for i, (ph0, u0, v0, prm) in enumerate(inst):
        n = specs[i]["n"]
        with bf.Grid(n) as g:
            t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
            ph, pp, uu, vv = t(ph0), g.field(0.0), g.field(0.0), g.field(0.0)
            g.step(bf.make_params(**prm), ph, t(u0), t(v0), pp, uu, vv,
                   bf.default_opts(bf.OP_CH, rtol=1e-10), bf.default_opts(bf.OP_LAP, rtol=1e-12))
            torch.cuda.synchronize()
            assert relw(unpack(ens, phi, i), ph.cpu().numpy()) <= 1e-11
            assert relw(unpack(ens, p, i), pp.cpu().numpy()) <= 1e-10


def test_ensemble_largest_instance_size(dev):
    """An 8192 x 8192 instance (the largest size an ensemble accepts) next to
    a 128 x 128 one: the large instance against the single-grid step of the
    same state, the small one against the oracle."""
    specs = S.ensemble_specs(2, seed=31, sizes=(128,))
    specs[0]["n"] = 8192
    print("ensemble 8192 + 128", flush=True)
    ens, inst, phi, p, u, v, stats, ms = run(specs, dev)
    for sc, sp in stats[0]:
        assert sc.status in (bf.OK, bf.AT_FLOOR) and sp.status == bf.OK
    ph0, u0, v0, prm = inst[0]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    with bf.Grid(8192) as g:
        ph, pp, uu, vv = t(ph0), g.field(0.0), g.field(0.0), g.field(0.0)
        g.step(bf.make_params(**prm), ph, t(u0), t(v0), pp, uu, vv,
               bf.default_opts(bf.OP_CH, rtol=1e-10), bf.default_opts(bf.OP_LAP, rtol=1e-12))
        torch.cuda.synchronize()
        e = (relw(unpack(ens, phi, 0), ph.cpu().numpy()), relw(unpack(ens, p, 0), pp.cpu().numpy()),
             relw(unpack(ens, u, 0), uu.cpu().numpy()))
    print(f"step {ms:.1f} ms, 8192 instance vs single grid {e}", flush=True)
    assert e[0] <= 1e-10 and e[1] <= 1e-10 and e[2] <= 1e-10
    ph0, u0, v0, prm = inst[1]
    rphi, rp, ru, rv = oracle.step.step(ph0, u0, v0, **prm)
    assert relw(unpack(ens, phi, 1), rphi) <= 1e-10
    assert relw(unpack(ens, p, 1), rp) <= 1e-10


def test_ensemble_rejects_bad_parameters_and_options(dev):
    """Per-instance parameters and the solver options are checked before any
    work is queued; the fields are left as they were."""
    ens = bf.Ensemble([128, 256])
    phi = ens.field(0.25)
    z = ens.field(0.0)
    good = bf.make_params(**S.DEFAULT_PARAMS)
    bad = bf.make_params(**dict(S.DEFAULT_PARAMS, dt=0.0))
    with pytest.raises(bf.BiofilmError, match="EINVAL"):
        ens.step([good, bad], phi, z, z, ens.field(0.0))
    with pytest.raises(bf.BiofilmError, match="EUNSUPPORTED"):
        ens.step([good, good], phi, z, z, ens.field(0.0),
                 ch=bf.default_opts(bf.OP_CH, mg_precision=bf.MG_F32))
    with pytest.raises(bf.BiofilmError, match="EUNSUPPORTED"):
        ens.step([good, good], phi, z, z, ens.field(0.0),
                 pr=bf.default_opts(bf.OP_LAP, ksp=bf.KSP_GMRES))
    with pytest.raises(ValueError):
        ens.step([good], phi, z, z, ens.field(0.0))
    torch.cuda.synchronize()
    assert bool(torch.all(phi == 0.25))


def test_ensemble_step_depends_only_on_its_arguments(dev):
    """An ensemble keeps nothing between steps: the same states stepped again
    after a step from other states (and with other values in the output
    arrays) give bit-identical fields and iteration counts."""
    specs = S.ensemble_specs(3, sizes=(128, 256))
    inst = [S.ensemble_instance(s) for s in specs]
    other = [S.ensemble_instance(dict(s, seed_phi=s["seed_phi"] + 500)) for s in specs]
    ens = bf.Ensemble([s["n"] for s in specs])
    prms = [bf.make_params(**a[3]) for a in inst]
    oc = bf.default_opts(bf.OP_CH, rtol=1e-10)
    op = bf.default_opts(bf.OP_LAP, rtol=1e-12)

    def one(states, fill):
        phi = pack(ens, [a[0] for a in states], dev)
        us = pack(ens, [a[1] for a in states], dev)
        vs = pack(ens, [a[2] for a in states], dev)
        p, u, v = ens.field(fill), ens.field(fill), ens.field(fill)
        st, _ = ens.step(prms, phi, us, vs, p, u, v, oc, op)
        torch.cuda.synchronize()
        return ([t.cpu().numpy() for t in (phi, p, u, v)],
                [(s.iters, s.restarts) for pair in st for s in pair])

    first, it1 = one(inst, 0.0)
    one(other, 0.0)
    again, it2 = one(inst, 2.0)
    assert it1 == it2
    for a, b in zip(first, again):
        assert np.array_equal(a, b)


def test_masked_instance_next_to_iterating_ones(dev):
    """Instance 1 has no flow: its pressure right-hand side is zero, so it is
    masked from the start and must come out as p = 0, u = v = 0, while its
    class mates solve normally."""
    specs = S.ensemble_specs(3, seed=9, sizes=(128,))
    ens, inst, phi, p, u, v, stats, _ = run(specs, dev, zero_flow=(1,))
    assert np.all(unpack(ens, p, 1) == 0) and np.all(unpack(ens, u, 1) == 0)
    assert stats[0][1][1].iters == 0 and stats[0][1][1].status == bf.OK
    for i in (0, 2):
        ph0, u0, v0, prm = inst[i]
        rphi, rp, ru, rv = oracle.step.step(ph0, u0, v0, **prm)
        assert relw(unpack(ens, p, i), rp) <= 1e-10
        assert relw(unpack(ens, phi, i), rphi) <= 1e-10


@pytest.mark.timeout(900)
def test_ensemble_configuration_64_instances_10_steps(dev):
    """The batched-ensemble configuration: 64 seeded instances of sizes in
    {128, 256, 512, 1024}, 10 steps; every solve ends OK / AT_FLOOR, and every
    instance is compared with 10 oracle steps of its own parameters."""
    specs = S.ensemble_specs(64)
    ens, inst, phi, p, u, v, stats, ms = run(specs, dev, steps=10)
    print("classes", ens.info(), f"last step {ms:.1f} ms")
    bad = [(k, i, sc, sp) for k, st in enumerate(stats) for i, (sc, sp) in enumerate(st)
           if sc.status not in (bf.OK, bf.AT_FLOOR) or sp.status != bf.OK]
    for k, i, sc, sp in bad[:5]:
        print(f"  step {k} inst {i} n={specs[i]['n']}: CH {sc}  P {sp}")
    assert not bad
    its = [sc.iters for st in stats for sc, _ in st]
    print(f"  CH iterations {min(its)}..{max(its)}, restarts "
          f"{sum(sc.restarts for st in stats for sc, _ in st)}")
    worst = {}
    with scipy.fft.set_workers(WORKERS):
        for i, s in enumerate(specs):
            ph0, u0, v0, prm = inst[i]
            rphi, rp, ru, rv = oracle.step.run(ph0, u0, v0, 10, **prm)
            e = (relw(unpack(ens, phi, i), rphi), relw(unpack(ens, p, i), rp),
                 relw(unpack(ens, u, i), ru), relw(unpack(ens, v, i), rv))
            worst[s["n"]] = max(worst.get(s["n"], 0.0), max(e))
            assert max(e) <= 1e-10, (i, s, e)
    print("  worst error after 10 steps per size (phi, p, u, v): "
          + ", ".join(f"{n}: {w:.1e}" for n, w in sorted(worst.items())))
    assert len(worst) == 4
