"""Benchmark: biofilm-flow time step on one MI355X.

A step is the whole hot path over one 4096 x 4096 grid with float64 fields:
the Flory-Huggins right-hand side, the Cahn-Hilliard solve (13-point
operator, MG-preconditioned CG to rtol 1e-10, stopping at the float64 floor),
the pressure right-hand side, the pressure Poisson solve (5-point operator,
MG-preconditioned CG to rtol 1e-12, where p meets the 1e-10 forward-error bar)
and the velocity correction.  Inputs are
synthetic (seeded initial biofilm and inflow) and resident in HBM before the
timed region.

Two precisions are timed over the same K steps from the same initial state:
mixed (float32 multigrid V-cycle inside float64 CG, float64 residuals,
iterate and step arithmetic) and plain float64.  `value` is the mixed
device time per step (ms, lower is better); `fp64_ms_per_step` is the
float64 one at the same tolerance, and `mixed_vs_fp64_rel_diff` the weighted
relative difference of the two final states.

`roofline` covers the 13-point stencil SpMV (y = x + c L^2 x, float64) timed
with HIP events on the grid's stream over back-to-back launches on rotating
buffers (so the 256 MB last-level cache cannot hold the working set).
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 4096]
       [--precision both|mixed|f64] [--no-cpu-baseline] [--spmv-only]
       [--steps-only]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1811_11842_amd as bf  # noqa: E402
import synthetic as S  # noqa: E402

METRIC = "solve time/step + stencil SpMV HBM GB/s at 4096², mixed vs FP64 @1e-10"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1811_11842_amd/csrc/stream.hip", "paper_1811_11842_amd/csrc/stencil_ops.hpp",
                  "paper_1811_11842_amd/csrc/common.hpp", "paper_1811_11842_amd/csrc/kernels.hip"]
# HBM traffic per launch at 4096^2 from `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
# (profiles/spmv_13pt_4096_counters.md for the SpMV and the sweep,
# profiles/step_kernels_4096_counters.md for the CG step), KiB per dispatch, scaled by the ratio of known to
# counted bytes of the bf_copy calibration kernel.  Valid only for the kernel sources
# whose sha256 is recorded; otherwise the traffic is reported as null.
TRAFFIC_RECORD = {"n": 4096, "fetch_scale": 1.9996, "write_scale": 1.0, "kernels": {"spmv": {"fetch_kib": 69688.0, "write_kib": 131104.0}, "smooth": {"fetch_kib": 200794.4, "write_kib": 131104.0}, "cg_step": {"fetch_kib": 103494.7, "write_kib": 202005.7}, "r_update": {"fetch_kib": 131120.5, "write_kib": 196688.1}}, "sources_sha256": "0b674dcfa35ae61826fa492e474ab23a78ca3361c59ee3d611f60eaac372ee6d"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--precision", choices=["both", "mixed", "f64"], default="both")
    ap.add_argument("--ensemble", action="store_true",
                    help="time only the batched ensemble (64 instances, 10 steps)")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--spmv-reps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--spmv-only", action="store_true")
    ap.add_argument("--steps-only", action="store_true")
    ap.add_argument("--smooth-only", action="store_true",
                    help="only time the smoothing sweep (for profiling that kernel)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain device copy of one field (for HBM counter calibration)")
    ap.add_argument("--leg", choices=["predictor", "mobility", "cn", "adjoint"],
                    help="only time one of the variant legs (for profiling it)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Relative residual of the pressure solves: at 1e-10 the 4096^2 pressure
# forward error against the oracle is 1.00e-10 (the low Laplacian modes keep
# what the residual leaves), at 1e-12 it is 3.3e-12 for one more iteration,
# so the step meets the 1e-10 forward-error bar on p as it does on phi.
PRESSURE_RTOL = 1e-12

# The live timing of the CG step and the residual update records HIP events
# around every 8th launch (each event leaves the stream idle for a few
# microseconds; 20 steps give about 34 samples of each kernel).
CG_TIMING_EVERY = 8


def time_steps(g, n, steps, warmup, mg_precision):
    """Warm up on a copy of the initial state, then time `steps` steps from
    the initial state itself; returns device ms/step, wall ms/step, stats and
    the final (phi, p)."""
    dev = g.device
    phi0 = S.initial_phi(n)
    u0, v0 = S.inflow_velocity(n)
    prm = bf.make_params(**S.DEFAULT_PARAMS)
    phi = torch.from_numpy(phi0).to(dev)
    us, vs = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
    p, u, v = g.field(0.0), g.field(0.0), g.field(0.0)
    oc = bf.default_opts(bf.OP_CH, rtol=1e-10, mg_precision=mg_precision)
    op = bf.default_opts(bf.OP_LAP, rtol=PRESSURE_RTOL, mg_precision=mg_precision)
    phw = phi.clone()
    for k in range(warmup):
        st = g.step(prm, phw, us, vs, p, u, v, oc, op)
        log(f"warmup step {k}: CH {st[0].as_dict()} P {st[1].as_dict()}")
    del phw
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stats = []
    g.cg_timing(CG_TIMING_EVERY)
    t0 = time.perf_counter()
    e0.record()
    for k in range(steps):
        st = g.step(prm, phi, us, vs, p, u, v, oc, op)
        stats.append(st)
        log(f"step {k}: CH it={st[0].iters} {bf.STATUS_NAMES[st[0].status]} "
            f"res={st[0].rel_res_true:.2e} {st[0].ms:.2f} ms | P it={st[1].iters} "
            f"res={st[1].rel_res_true:.2e} {st[1].ms:.2f} ms")
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    cg = g.cg_timing_read()
    ru = g.rupdate_timing_read()
    g.cg_timing(False)
    return ms / steps, wall / steps * 1e3, stats, (phi, p), (cg, ru)


# Algorithmic bytes per grid point of the Cahn-Hilliard CG step kernel: z and
# p_old read, p' and q written, and x read and written for its deferred update.
# z and the search directions p are float32 with the float32 V-cycle, float64
# otherwise; q and x are float64.  The first step of a Krylov cycle reads z
# only and writes p' and q.  With the float32 V-cycle on grids up to 8192^2 the
# library keeps the directions of up to 16 steps and updates x in one separate
# pass per batch (k_x_accum), so the step itself does not touch x.
def cg_step_bytes(z_bytes, launches, first, x_in_step=True):
    p_bytes = z_bytes
    xb = 16 if x_in_step else 0
    return ((launches - first) * (z_bytes + 2 * p_bytes + 8 + xb)
            + first * (z_bytes + p_bytes + 8))


def x_in_cg_step(n, mg_precision):
    """False where the library updates x in batches (float32 V-cycle, at least
    three float32 fields of (n+1) n nodes within 1 GiB)."""
    if os.environ.get("BF_NO_RING") == "1":
        return True
    return not (mg_precision == bf.MG_F32 and 3 * 4 * (n + 1) * n <= 2 ** 30)


# Algorithmic bytes per grid point of the residual update: r and q read, r
# written (float64), and with the float32 V-cycle its float32 copy of r.
def ru_roofline(n, ru, mixed, kernel, traffic):
    total_ms, launches = ru
    npts = (n + 1) * n
    alg = (28 if mixed else 24) * npts
    us = total_ms / launches * 1e3
    gbs = alg / (us * 1e-6) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes": int(alg), "launch_us": round(us, 3), "launches": launches,
            "timing": f"HIP events on the grid's stream around every {CG_TIMING_EVERY}th launch "
                      "in the Cahn-Hilliard solves of the timed steps"}


def cg_roofline(n, cg, z_bytes, kernel, traffic, x_in_step=True):
    total_ms, launches, first = cg
    npts = (n + 1) * n
    alg = cg_step_bytes(z_bytes, launches, first, x_in_step) * npts / launches
    us = total_ms / launches * 1e3
    gbs = alg / (us * 1e-6) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes": int(alg), "launch_us": round(us, 3), "launches": launches,
            "first_launches": first,
            "timing": f"HIP events on the grid's stream around every {CG_TIMING_EVERY}th launch "
                      "in the timed steps"}


def wrel(a, b):
    """||a - b||_W / ||b||_W (trapezoid weights in y) on the device."""
    w = torch.ones(a.shape[0], 1, dtype=a.dtype, device=a.device)
    w[0] = w[-1] = 0.5
    return float(torch.sqrt((w * (a - b) ** 2).sum() / (w * b ** 2).sum()))


def step_summary(prefix, ms_step, wall_ms, stats):
    it_ch = [s[0].iters for s in stats]
    it_p = [s[1].iters for s in stats]
    return {
        f"{prefix}ms_per_step": round(ms_step, 4),
        f"{prefix}wall_ms_per_step": round(wall_ms, 4),
        f"{prefix}ch_iters_mean": float(np.mean(it_ch)),
        f"{prefix}p_iters_mean": float(np.mean(it_p)),
        f"{prefix}ch_solve_ms_mean": round(float(np.mean([s[0].ms for s in stats])), 4),
        f"{prefix}p_solve_ms_mean": round(float(np.mean([s[1].ms for s in stats])), 4),
        f"{prefix}ch_status": sorted({bf.STATUS_NAMES[s[0].status] for s in stats}),
        f"{prefix}p_status": sorted({bf.STATUS_NAMES[s[1].status] for s in stats}),
        f"{prefix}ch_rel_res_true_max": float(max(s[0].rel_res_true for s in stats)),
        f"{prefix}p_rel_res_true_max": float(max(s[1].rel_res_true for s in stats)),
    }


def time_spmv(g, n, reps):
    """Average duration of the 13-point operator kernel over `reps` launches."""
    dev = g.device
    nbuf = 4
    xs = [torch.from_numpy(S.random_field(n, 50 + k)).to(dev) for k in range(nbuf)]
    ys = [g.field() for _ in range(nbuf)]
    c = S.DEFAULT_PARAMS["dt"] * S.DEFAULT_PARAMS["M"] * S.DEFAULT_PARAMS["kappa"]
    for k in range(nbuf):
        g.apply(bf.OP_CH, c, xs[k], ys[k])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        g.apply(bf.OP_CH, c, xs[r % nbuf], ys[r % nbuf])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_copy(g, n, reps):
    """Average duration of the library's plain copy of one field (bf_copy: 16-byte
    lanes, coalesced rows, ordinary loads and stores) on 4 rotating buffer pairs: the
    ceiling of a kernel that reads one field and writes one."""
    dev = g.device
    xs = [torch.from_numpy(S.random_field(n, 90 + k)).to(dev) for k in range(4)]
    ys = [g.field() for _ in range(4)]
    for k in range(4):
        g.copy(xs[k], ys[k])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        g.copy(xs[r % 4], ys[r % 4])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_smooth(g, n, reps):
    """Average duration of one Cahn-Hilliard smoothing sweep (x, x_prev, b -> x')."""
    dev = g.device
    nset = 2
    sets = [[torch.from_numpy(S.random_field(n, 70 + 4 * k + m)).to(dev) for m in range(4)]
            for k in range(nset)]
    c = S.DEFAULT_PARAMS["dt"] * S.DEFAULT_PARAMS["M"] * S.DEFAULT_PARAMS["kappa"]
    for x, xp, b, out in sets:
        g.smooth(bf.OP_CH, c, x, b, out, xp, 0.4, 0.3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        x, xp, b, out = sets[r % nset]
        g.smooth(bf.OP_CH, c, x, b, out, xp, 0.4, 0.3)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_ensemble(steps=10, warmup=1, count=64):
    """The batched-ensemble configuration (64 seeded instances of sizes in
    {128, 256, 512, 1024} with their own chi, dt, radius and noise, float64):
    device time per ensemble step, and the same instances stepped one after
    the other on single grids (the unbatched path) for comparison."""
    specs = S.ensemble_specs(count)
    inst = [S.ensemble_instance(sp) for sp in specs]
    dev = torch.device("cuda", torch.cuda.current_device())
    ens = bf.Ensemble([sp["n"] for sp in specs])

    def pack(arrays):
        t = torch.zeros(ens.total, dtype=torch.float64)
        for i, a in enumerate(arrays):
            o = ens.offsets[i]
            t[o:o + a.size] = torch.from_numpy(np.ascontiguousarray(a).ravel())
        return t.to(dev)

    phi0 = pack([a[0] for a in inst])
    us, vs = pack([a[1] for a in inst]), pack([a[2] for a in inst])
    p, u, v = ens.field(0.0), ens.field(0.0), ens.field(0.0)
    prms = [bf.make_params(**a[3]) for a in inst]
    oc, op = bf.default_opts(bf.OP_CH, rtol=1e-10), bf.default_opts(bf.OP_LAP, rtol=PRESSURE_RTOL)
    phi = phi0.clone()
    for _ in range(warmup):
        ens.step(prms, phi, us, vs, p, u, v, oc, op)
    phi.copy_(phi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = 0
    its = []
    dev_ms = 0.0
    for _ in range(steps):
        st, ms = ens.step(prms, phi, us, vs, p, u, v, oc, op)  # ms: HIP events of the step
        dev_ms += ms
        worst = max(worst, max(max(a.status, b.status) for a, b in st))
        its.append(sum(a.iters for a, _ in st) / count)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) / steps * 1e3
    ens_ms = dev_ms / steps
    # unbatched: every instance on its own grid, one after the other
    seq_ms = 0.0
    for sp, (ph, uu, vv, prm) in zip(specs, inst):
        with bf.Grid(sp["n"]) as g:
            t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
            x, us1, vs1 = t(ph), t(uu), t(vv)
            p1, u1, v1 = g.field(0.0), g.field(0.0), g.field(0.0)
            P = bf.make_params(**prm)
            xw = x.clone()
            for _ in range(warmup):
                g.step(P, xw, us1, vs1, p1, u1, v1, oc, op)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                g.step(P, x, us1, vs1, p1, u1, v1, oc, op)
            e1.record()
            torch.cuda.synchronize()
            seq_ms += e0.elapsed_time(e1) / steps
    points = sum((sp["n"] + 1) * sp["n"] for sp in specs)
    classes = [{"n": c[0], "instances": c[1], "tile_rows": c[2]} for c in ens.info()]
    ens.close()
    return {"instances": count, "steps": steps, "points": points, "classes": classes,
            "ms_per_step": round(ens_ms, 3), "wall_ms_per_step": round(wall_ms, 3),
            "sequential_ms_per_step": round(seq_ms, 3),
            "speedup_vs_sequential": round(seq_ms / ens_ms, 2),
            "ch_iters_mean": round(float(np.mean(its)), 2),
            "worst_status": bf.STATUS_NAMES.get(worst, str(worst)),
            "timing": "HIP events per step on the caller's stream (start marker every size class "
                      "waits for, end marker waiting for every class); the one-by-one leg: HIP "
                      "events around each instance's steps"}


def time_cn(g, n, steps=5):
    """Crank-Nicolson Cahn-Hilliard steps (bf_step_ch_cn, float64, rtol 1e-10)."""
    phi = torch.from_numpy(S.initial_phi(n)).to(g.device)
    prev = g.field(0.0)
    prm = bf.make_params(**S.DEFAULT_PARAMS)
    o = bf.default_opts(bf.OP_CH, rtol=1e-10)
    g.step_ch_cn(prm, phi, prev, first=True, opts=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(steps):
        its.append(g.step_ch_cn(prm, phi, prev, first=False, opts=o).iters)
    torch.cuda.synchronize()
    return {"n": n, "steps": steps, "ms_per_step": round((time.perf_counter() - t0) / steps * 1e3, 3),
            "ch_iters_mean": float(np.mean(its))}


def time_predictor(g, n, calls=5):
    """Momentum predictor (bf_momentum_predict: explicit advection, Crank-
    Nicolson viscous term at the paper's viscous scale nu = 1e3, dt = 1e-4,
    two Helmholtz solves at rtol 1e-12 run concurrently), float64 and
    float32-V-cycle multigrid: wall time per call."""
    Y, X = S.node_coords(n)
    u0, v0 = S.inflow_velocity(n, U=0.1)
    u0 = u0 + 0.05 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y)
    v0 = v0 + 0.05 * np.cos(2 * np.pi * X) * np.sin(np.pi * Y) ** 2
    u0[0], u0[-1], v0[0], v0[-1] = 0.0, 0.1, 0.0, 0.0
    u = torch.from_numpy(u0).to(g.device)
    v = torch.from_numpy(v0).to(g.device)
    us, vs = g.field(0.0), g.field(0.0)
    res = {"n": n, "dt": 1e-4, "nu": 1e3, "theta": 0.5, "rtol": 1e-12}
    for name, mp in (("f64", bf.MG_F64), ("mixed", bf.MG_F32)):
        o = bf.default_opts(bf.OP_HELM, rtol=1e-12, mg_precision=mp)
        g.momentum_predict(1e-4, 1e3, 0.5, 0.1, u, v, us, vs, opts=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for _ in range(calls):
            _, _, (su, sv) = g.momentum_predict(1e-4, 1e3, 0.5, 0.1, u, v, us, vs, opts=o)
            its.append((su.iters, sv.iters))
        torch.cuda.synchronize()
        res[f"{name}_ms_per_call"] = round((time.perf_counter() - t0) / calls * 1e3, 3)
        res[f"{name}_iters"] = [float(np.mean([a for a, _ in its])), float(np.mean([b for _, b in its]))]
    return res


def time_mobility(g, n, steps=3):
    """Cahn-Hilliard steps with the phi-dependent mobility (bf_step_ch_mob:
    GMRES(10) preconditioned by the constant-mobility float32 V-cycle, rtol
    1e-10): wall time per step."""
    phi = torch.from_numpy(S.initial_phi(n)).to(g.device)
    prm = bf.make_params(**S.DEFAULT_PARAMS)
    o = bf.default_opts(bf.OP_CH, ksp=bf.KSP_GMRES, restart=10, mg_precision=bf.MG_F32)
    g.step_ch_mob(prm, phi, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, sts = [], []
    for _ in range(steps):
        st = g.step_ch_mob(prm, phi, o)
        its.append(st.iters)
        sts.append(st.status)
    torch.cuda.synchronize()
    return {"n": n, "steps": steps, "ms_per_step": round((time.perf_counter() - t0) / steps * 1e3, 3),
            "gmres_iters_mean": float(np.mean(its)),
            "status": sorted({bf.STATUS_NAMES.get(s, str(s)) for s in sts})}


def time_adjoint(n=2048, steps=20, every=5):
    """Gradient of the upper-half mass after `steps` advected Cahn-Hilliard
    steps with respect to phi0, chi and the inflow speed (checkpoints every
    `every` steps): wall time of the forward and of the reverse pass."""
    from paper_1811_11842_amd import adjoint as bfa
    dev = torch.device("cuda", torch.cuda.current_device())
    Y, _ = S.node_coords(n)
    nu, nv = S.inflow_velocity(n, U=0.0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    prm = {k: S.DEFAULT_PARAMS[k] for k in ("dt", "M", "kappa", "Npoly")}
    with bf.Grid(n) as g:
        ro = bfa.Rollout(g, steps, t(Y * (2.0 - Y)), t(nu), t(nv), checkpoint_every=every,
                         rtol_forward=1e-12, rtol_adjoint=1e-12, rtol_pressure=1e-12, **prm)
        p0 = t(S.initial_phi(n)).requires_grad_(True)
        chi = torch.tensor(S.DEFAULT_PARAMS["chi"], dtype=torch.float64, requires_grad=True)
        U = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
        w = bfa.upper_half_weights(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = (w * bfa.RolloutFn.apply(p0, chi, U, ro)).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    return {"n": n, "steps": steps, "checkpoint_every": every, "J": J.item(),
            "dJ_dchi": chi.grad.item(), "dJ_dU": U.grad.item(),
            "forward_ms": round((t1 - t0) * 1e3, 1), "reverse_ms": round((t2 - t1) * 1e3, 1)}


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kernel, n):
    rec = TRAFFIC_RECORD
    if not rec or rec.get("n") != n or rec.get("sources_sha256") != sources_sha256():
        return None
    k = rec["kernels"].get(kernel)
    if not k:
        return None
    return int(k["fetch_kib"] * 1024 * rec["fetch_scale"] + k["write_kib"] * 1024 * rec["write_scale"])


def cpu_threads():
    """Host threads this process may use (its affinity set, at most 16: the
    CPU share of one GPU on the measurement hosts)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, steps, workers):
    """Oracle steps at n x n (numpy/scipy float64, spectral solves), timed as
    the oracle stands, with scipy.fft using `workers` threads."""
    import scipy.fft
    import oracle  # the CPU oracle, timed as it stands
    phi = S.initial_phi(n)
    u, v = S.inflow_velocity(n)
    with scipy.fft.set_workers(workers):
        t0 = time.perf_counter()
        for _ in range(steps):
            phi, p, uu, vv = oracle.step.step(phi, u, v, **S.DEFAULT_PARAMS)
        dt = time.perf_counter() - t0
    return dt / steps * 1e3


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    n = a.n
    npts = (n + 1) * n
    if a.copy_calib:
        # plain copy kernels of known size: each reads 8*npts bytes and writes
        # 8*npts bytes, rotating over 4 buffer pairs (1 GB): the library's
        # bf_copy (16-byte lanes, the access pattern of the stencil kernels)
        # and, for comparison, the runtime's copy
        xs = [torch.rand(n + 1, n, dtype=torch.float64, device="cuda") for _ in range(4)]
        ys = [torch.empty_like(xs[0]) for _ in range(4)]
        torch.cuda.synchronize()
        with bf.Grid(n) as g:
            for r in range(20):
                g.copy(xs[r % 4], ys[r % 4])
            torch.cuda.synchronize()
            assert torch.equal(ys[0], xs[0])
            for r in range(20):
                ys[r % 4].copy_(xs[r % 4])
            torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_each_way": 8 * npts, "launches": 20}), flush=True)
        return
    out = {"metric": METRIC, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic"}
    if a.ensemble:
        print(json.dumps({"ensemble": time_ensemble()}), flush=True)
        return
    if a.leg:
        if a.leg == "adjoint":
            res = time_adjoint()
        else:
            with bf.Grid(n) as g:
                res = {"predictor": time_predictor, "mobility": time_mobility,
                       "cn": time_cn}[a.leg](g, n)
        print(json.dumps({a.leg: res}), flush=True)
        return
    with bf.Grid(n) as g:
        if a.smooth_only:
            t_sm = time_smooth(g, n, a.spmv_reps)
            print(json.dumps({"smooth_us": round(t_sm * 1e3, 3),
                              "smooth_gbs": round(32 * npts / (t_sm * 1e-3) / 1e9, 1)}), flush=True)
            return
        if not a.spmv_only:
            res = {}
            if a.precision in ("both", "mixed"):
                ms_m, wall_m, st_m, fin_m, (cg_m, ru_m) = time_steps(g, n, a.steps, a.warmup,
                                                                     bf.MG_F32)
                res["mixed"] = fin_m
                out.update({"value": round(ms_m, 4), "unit": "ms/step",
                            "ms_per_step": round(ms_m, 4)})
                out.update(step_summary("", ms_m, wall_m, st_m))
                # the kernel with the largest share of the step's time: the residual
                # update of both solves' iterations (timed in the Cahn-Hilliard solve)
                out["roofline_step"] = ru_roofline(
                    n, ru_m, True, "k_r_update (residual update of the value's steps: r -= alpha q, "
                    "||r||^2 partials, float32 copy of r)", recorded_traffic("r_update", n))
                out["roofline_cg_step"] = cg_roofline(
                    n, cg_m, 4, "k_cg_ch<4,float,4> (Cahn-Hilliard CG step of the value's "
                    "steps: p' = z + beta p, q = A p' exactly rounded, <p', q>_W; z and p float32"
                    + ("; x += alpha p" if x_in_cg_step(n, bf.MG_F32) else
                       "; x updated in batches of up to 16 steps by k_x_accum") + ")",
                    recorded_traffic("cg_step", n), x_in_cg_step(n, bf.MG_F32))
            if a.precision in ("both", "f64"):
                ms_d, wall_d, st_d, fin_d, (cg_d, ru_d) = time_steps(g, n, a.steps, a.warmup,
                                                                     bf.MG_F64)
                res["f64"] = fin_d
                out["fp64_roofline_step"] = ru_roofline(
                    n, ru_d, False, "k_r_update (the same update without the float32 copy)", None)
                out["fp64_roofline_cg_step"] = cg_roofline(
                    n, cg_d, 8, "k_cg_ch<4,double,4> (the same step with float64 z and p)", None)
                if a.precision == "f64":
                    out.update({"value": round(ms_d, 4), "unit": "ms/step",
                                "ms_per_step": round(ms_d, 4)})
                out.update(step_summary("fp64_", ms_d, wall_d, st_d))
            if len(res) == 2:
                out["speedup_mixed_vs_fp64"] = round(out["fp64_ms_per_step"] / out["ms_per_step"], 3)
                out["mixed_vs_fp64_rel_diff"] = {
                    "phi": wrel(res["mixed"][0], res["f64"][0]),
                    "p": wrel(res["mixed"][1], res["f64"][1])}
            out["dtype"] = {"both": "f64+f32", "mixed": "f64+f32", "f64": "f64"}[a.precision]
        if not a.steps_only:
            t_spmv = time_spmv(g, n, a.spmv_reps)
            alg = 16 * npts      # algorithmic: read x once, write y once (float64)
            gbs = alg / (t_spmv * 1e-3) / 1e9
            out["spmv_us"] = round(t_spmv * 1e3, 3)
            out["spmv_gbs"] = round(gbs, 1)
            t_copy = time_copy(g, n, a.spmv_reps)
            out["roofline"] = {"kernel": "k_stream<1,0,5,double,double> (13-point Cahn-Hilliard SpMV, float64, 5-row tiles)",
                               "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                               "traffic": recorded_traffic("spmv", n), "algorithmic_bytes": alg,
                               "launch_us": round(t_spmv * 1e3, 3),
                               "copy_us": round(t_copy * 1e3, 3),
                               "frac_of_copy": round(t_copy / t_spmv, 4)}
            if not a.spmv_only:
                t_sm = time_smooth(g, n, max(20, a.spmv_reps // 2))
                alg_sm = 32 * npts   # x, x_prev, b read, x' written
                gbs_sm = alg_sm / (t_sm * 1e-3) / 1e9
                out["roofline_smoother"] = {
                    "kernel": "k_stream<1,4,4,double,double> (13-point Chebyshev smoothing sweep, float64)",
                    "bound": "hbm", "achieved": round(gbs_sm, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs_sm / HBM_PEAK_GBS, 4),
                    "traffic": recorded_traffic("smooth", n), "algorithmic_bytes": alg_sm,
                    "launch_us": round(t_sm * 1e3, 3)}
    prec = {"both": "float32 V-cycle in float64 CG (value) and plain float64",
            "mixed": "float32 V-cycle in float64 CG", "f64": "plain float64"}[a.precision]
    out["config"] = {"workload": f"{n}x{n} grid, {a.steps} steps: Flory-Huggins RHS + MG-PCG "
                                 f"Cahn-Hilliard solve (rtol 1e-10) + MG-PCG pressure solve "
                                 f"(rtol {PRESSURE_RTOL:g}) + velocity correction, forward "
                                 f"error <= 1e-10, {prec}",
                     "ch_rtol": 1e-10, "pressure_rtol": PRESSURE_RTOL,
                     "precision": a.precision, "mg_precision_value": "f32" if a.precision != "f64" else "f64",
                     "n": n, "rows": n + 1, "cols": n, "points": npts,
                     "dt": S.DEFAULT_PARAMS["dt"], "kappa": S.DEFAULT_PARAMS["kappa"],
                     "chi": S.DEFAULT_PARAMS["chi"], "Npoly": S.DEFAULT_PARAMS["Npoly"]}
    if not (a.spmv_only or a.steps_only or a.smooth_only):
        with bf.Grid(n) as g:
            out["crank_nicolson"] = time_cn(g, n)
            log("momentum predictor (two Helmholtz solves)")
            out["momentum_predictor"] = time_predictor(g, n)
            log("variable-mobility Cahn-Hilliard steps")
            out["variable_mobility"] = time_mobility(g, n)
        out["adjoint"] = time_adjoint()
        log("float64 steps at 1024^2 (the plain float64 baseline configuration)")
        with bf.Grid(1024) as g1:
            ms1, _, st1, _, _ = time_steps(g1, 1024, 10, 2, bf.MG_F64)
        out["fp64_1024"] = {"n": 1024, "steps": 10, "ms_per_step": round(ms1, 4),
                            "ch_iters_mean": float(np.mean([s[0].iters for s in st1])),
                            "scaled_to_4096_ms": round(ms1 * 16, 3),
                            "note": "x16 points; measured 4096^2 float64 is fp64_ms_per_step"}
    if not (a.no_ensemble or a.spmv_only or a.steps_only or a.smooth_only):
        log("batched ensemble: 64 instances, 10 steps (and the same one by one)")
        out["ensemble"] = time_ensemble()
    if not a.no_cpu_baseline and not a.spmv_only:
        nt = cpu_threads()
        log(f"cpu baseline: {a.cpu_steps} oracle steps at {n}x{n}, {nt} FFT threads, then 2 "
            f"steps on one thread")
        cms = cpu_baseline(n, a.cpu_steps, nt)
        cms1 = cpu_baseline(n, 2, 1)
        out["cpu_baseline"] = {"value": round(cms, 1), "unit": "ms/step", "cores": nt,
                               "kind": "oracle",
                               "sample": f"{a.cpu_steps} oracle steps at {n}x{n} from the "
                                         f"benchmark's initial state (numpy/scipy float64, "
                                         f"spectral solves; scipy.fft on {nt} threads, numpy "
                                         f"elementwise work on one)",
                               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                               "one_thread_ms_per_step": round(cms1, 1)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
