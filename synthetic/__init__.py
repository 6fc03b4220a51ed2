"""Seeded synthetic workloads for the biofilm-flow time step.

This module is shared by the test harness, the benchmark and the CPU checker.
It holds the *workload recipe* only (geometry of the initial biofilm, inflow
profile, noise, seeds, parameter sets); none of the method's arithmetic
(operators, chemical potential, solves) lives here.  Both sides of every
comparison receive the same arrays produced by these functions; the GPU never
draws random numbers.

Workload (stand-in for the two-protrusion detachment run of Sec. 5.1, whose
inputs are not published): a biofilm base layer y < 0.2 and one protrusion, a
disc of radius r centred at (0.5, 0.2) unioned with the base (so the part
above the base is a half disc), volume fraction 0.3 inside, 0.02 outside,
plus seeded uniform noise and a clamp into (0, 1).  The flow is a shear
inflow u = U*y*(2 - y) (zero at the no-slip bottom wall, U at the top, cf. the
top shear of Sec. 5.1) plus seeded noise on interior rows.

Grid convention (Sec. 4: nodes (i*dx, j*dy); periodic x; no-flux y):
N intervals per side, h = 1/N, arrays of shape (N+1, N) indexed [j, i],
row-major with x fastest.  Column i = N is the periodic image of i = 0 and is
not stored.
"""
from __future__ import annotations

import numpy as np

# Parameter set of the reduced semi-implicit step (dimensionless).
DEFAULT_PARAMS = dict(dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6,
                      phi_lo=1e-6, phi_hi=1.0 - 1e-6)

SEED_PHI, SEED_U, SEED_V = 0, 1, 2


def grid_shape(n: int) -> tuple[int, int]:
    """(rows, cols) = (N+1, N) for N intervals per side."""
    return n + 1, n


def node_coords(n: int):
    """x = i/N (i = 0..N-1), y = j/N (j = 0..N), as float64 arrays (Y, X)."""
    x = np.arange(n, dtype=np.float64) / n
    y = np.arange(n + 1, dtype=np.float64) / n
    return np.meshgrid(y, x, indexing="ij")


def initial_phi(n: int, seed: int = SEED_PHI, radius: float = 0.1,
                base: float = 0.2, inside: float = 0.3, outside: float = 0.02,
                noise: float = 0.005, lo: float = 1e-6,
                hi: float = 1.0 - 1e-6) -> np.ndarray:
    """Seeded bimodal volume-fraction field, shape (N+1, N), float64."""
    Y, X = node_coords(n)
    inside_mask = (Y < base) | ((X - 0.5) ** 2 + (Y - base) ** 2 < radius ** 2)
    phi = np.where(inside_mask, inside, outside)
    rng = np.random.default_rng(seed)
    phi = phi + rng.uniform(-noise, noise, size=(n + 1, n))
    return np.clip(phi, lo, hi)


def inflow_velocity(n: int, U: float = 1.0, noise: float = 1e-3,
                    seed_u: int = SEED_U, seed_v: int = SEED_V):
    """Provisional velocity (u*, v*), each (N+1, N) float64.

    u* = U*y*(2-y) + noise, v* = noise; noise only on interior rows
    j = 1..N-1, wall rows exact (v* = 0 on both walls).
    """
    Y, _ = node_coords(n)
    u = U * Y * (2.0 - Y)
    v = np.zeros((n + 1, n))
    ru = np.random.default_rng(seed_u).uniform(-noise, noise, size=(n + 1, n))
    rv = np.random.default_rng(seed_v).uniform(-noise, noise, size=(n + 1, n))
    u[1:-1] += ru[1:-1]
    v[1:-1] += rv[1:-1]
    return u, v


def random_field(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Plain U(-scale, scale) field, shape (N+1, N), for operator tests."""
    return np.random.default_rng(seed).uniform(-scale, scale, size=(n + 1, n))


# Workload configurations: sizes, step counts, tolerances.
CONFIGS = {
    "small_64": dict(n=64, steps=1, rtol=1e-12),
    "plain_1024": dict(n=1024, steps=50, rtol=1e-10),
    "large_4096": dict(n=4096, steps=20, rtol=1e-10),
}


SEED_ENSEMBLE = 7


def ensemble_specs(count: int = 64, seed: int = SEED_ENSEMBLE,
                   sizes=(128, 256, 512, 1024)) -> list[dict]:
    """Seeded batched-ensemble recipe: per instance a size drawn uniformly
    from `sizes`, chi ~ U[0.5, 0.9], dt ~ U[5e-5, 2e-4], protrusion radius
    ~ U[0.05, 0.15] and its own noise seeds (other parameters as
    DEFAULT_PARAMS)."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(count):
        specs.append(dict(
            n=int(rng.choice(sizes)),
            chi=float(rng.uniform(0.5, 0.9)),
            dt=float(rng.uniform(5e-5, 2e-4)),
            radius=float(rng.uniform(0.05, 0.15)),
            seed_phi=1000 + 3 * k, seed_u=1001 + 3 * k, seed_v=1002 + 3 * k))
    return specs


def ensemble_instance(spec: dict):
    """(phi0, u*, v*, params) of one ensemble instance."""
    n = spec["n"]
    phi = initial_phi(n, seed=spec["seed_phi"], radius=spec["radius"])
    u, v = inflow_velocity(n, seed_u=spec["seed_u"], seed_v=spec["seed_v"])
    prm = dict(DEFAULT_PARAMS, chi=spec["chi"], dt=spec["dt"])
    return phi, u, v, prm
