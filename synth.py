"""Seeded synthetic inputs shared by the oracle side and the GPU side of the tests and the bench.

Holds none of the method's arithmetic: only random particle clouds, random potentials and the
configuration tables of the workloads. Everything is drawn from numpy's PCG64 with an explicit
seed, so the same call gives the same arrays on every machine.
"""
from __future__ import annotations

import numpy as np

# Workloads (box in Mpc/h; particles, fine mesh and coarse cells per side). The schedules are
# uniform in a (spacing 1): with a fixed step count this keeps the per-step drift roughly constant
# in the linear regime, above the resolution of 1-byte positions.
WORKLOADS = {
    "c1_pm32": dict(np_side=32, nm_side=64, nc_side=16, box=100.0, x_bytes=1, v_bytes=1,
                    omega_m=1.0, omega_l=0.0, h=0.7, sigma8=0.8, n_s=1.0,
                    a_init=0.02, a_final=1.0, n_steps=50, spacing=1, seed=1),
    "c2_pm128": dict(np_side=128, nm_side=256, nc_side=64, box=200.0, x_bytes=2, v_bytes=1,
                     omega_m=0.3, omega_l=0.7, h=0.7, sigma8=0.8, n_s=1.0,
                     a_init=0.02, a_final=1.0, n_steps=100, spacing=1, seed=2),
    "c3_pm2048": dict(np_side=2048, nm_side=2048, nc_side=512, box=2000.0, x_bytes=1, v_bytes=1,
                      omega_m=0.3, omega_l=0.7, h=0.7, sigma8=0.8, n_s=1.0,
                      a_init=0.02, a_final=1.0, n_steps=100, spacing=1, seed=3),
    # c3_pm2048's particle and cell resolution (64 particles per coarse cell) on a smaller box,
    # for profiling and kernel tuning
    "c3_density512": dict(np_side=512, nm_side=512, nc_side=128, box=500.0, x_bytes=1, v_bytes=1,
                          omega_m=0.3, omega_l=0.7, h=0.7, sigma8=0.8, n_s=1.0,
                          a_init=0.02, a_final=1.0, n_steps=100, spacing=1, seed=3),
    # same per-particle and per-cell resolution as c3_pm2048, small enough for the FP64 oracle
    "c3_sibling256": dict(np_side=256, nm_side=256, nc_side=64, box=250.0, x_bytes=1, v_bytes=1,
                          omega_m=0.3, omega_l=0.7, h=0.7, sigma8=0.8, n_s=1.0,
                          a_init=0.02, a_final=1.0, n_steps=100, spacing=1, seed=3),
}


def ensemble(seed: int = 4, nbox: int = 64, n_steps: int = 50) -> list[dict]:
    """Ensemble of independent boxes: particles per side drawn from {64, 96, 128, 192, 256}, a fine
    mesh of twice that per side, coarse cells a quarter of the mesh, 1.5625 Mpc/h per particle
    spacing, flat LCDM (Omega_m 0.3, h 0.7) with n_s ~ U[0.9, 1.0] and sigma8 ~ U[0.7, 0.9], 1-byte
    codes, Zel'dovich ICs at a = 0.02 with a seed per box, n_steps steps uniform in a to a = 1."""
    g = rng(seed)
    sides = g.choice([64, 96, 128, 192, 256], size=nbox)
    out = []
    for i, n in enumerate(sides):
        n = int(n)
        out.append(dict(np_side=n, nm_side=2 * n, nc_side=n // 2, box=1.5625 * n, x_bytes=1, v_bytes=1,
                        omega_m=0.3, omega_l=0.7, h=0.7, sigma8=float(g.uniform(0.7, 0.9)),
                        n_s=float(g.uniform(0.9, 1.0)), a_init=0.02, a_final=1.0, n_steps=n_steps, spacing=1,
                        seed=1000 + 17 * seed + i))
    return out


def ensemble_small(seed: int = 6, nbox: int = 64, side: int = 32, n_steps: int = 50) -> list[dict]:
    """Ensemble of equal small boxes (side^3 particles, mesh twice that per side, coarse cells a
    quarter of the mesh, 1.5625 Mpc/h per particle spacing), the same cosmology draws as ensemble:
    each box's kernels alone occupy a fraction of the GPU."""
    g = rng(seed)
    return [dict(np_side=side, nm_side=2 * side, nc_side=side // 2, box=1.5625 * side, x_bytes=1, v_bytes=1,
                 omega_m=0.3, omega_l=0.7, h=0.7, sigma8=float(g.uniform(0.7, 0.9)), n_s=float(g.uniform(0.9, 1.0)),
                 a_init=0.02, a_final=1.0, n_steps=n_steps, spacing=1, seed=2000 + 17 * seed + i)
            for i in range(nbox)]


def serving_jobs(seed: int = 5, n: int = 2000, rate: float = 20.0, n_steps: int = 50) -> list[dict]:
    """A Poisson stream of simulation requests: exponential gaps of mean 1/rate seconds; particles
    per side 64, 128 or 256 with probabilities 0.5, 0.35, 0.15; mesh twice and coarse cells half the
    particle count per side, 1.5625 Mpc/h per particle spacing; flat LCDM with sigma8 ~ U[0.7, 0.9];
    1-byte codes; n_steps steps to a = 1. Each item: dict(arrival=seconds, cfg=simulation parameters)."""
    g = rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    sides = g.choice([64, 128, 256], size=n, p=[0.5, 0.35, 0.15])
    out = []
    for i in range(n):
        side = int(sides[i])
        cfg = dict(np_side=side, nm_side=2 * side, nc_side=side // 2, box=1.5625 * side, x_bytes=1, v_bytes=1,
                   omega_m=0.3, omega_l=0.7, h=0.7, sigma8=float(g.uniform(0.7, 0.9)), n_s=1.0, a_init=0.02,
                   a_final=1.0, n_steps=n_steps, spacing=1, seed=50000 + i)
        out.append(dict(arrival=float(t[i]), cfg=cfg))
    return out


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def particle_cloud(seed: int, n: int, nm: int, vscale: float = 1.0, clump_frac: float = 0.25,
                   n_clumps: int = 4, clump_radius: float = 2.0):
    """Positions (n,3) in [0, nm) fine-mesh units and momenta (n,3).

    A uniform background plus a few Gaussian clumps (dense cells), and velocities made of a
    smooth bulk flow (so per-cell means are non-trivial) plus a Gaussian dispersion."""
    g = rng(seed)
    n_cl = int(n * clump_frac)
    x = g.uniform(0.0, nm, size=(n, 3))
    if n_cl and n_clumps:
        centres = g.uniform(0.0, nm, size=(n_clumps, 3))
        which = g.integers(0, n_clumps, size=n_cl)
        x[:n_cl] = centres[which] + g.normal(0.0, clump_radius, size=(n_cl, 3))
    x = np.mod(x, nm)
    x = np.where(x >= nm, 0.0, x)
    k = 2.0 * np.pi / nm
    phase = g.uniform(0, 2 * np.pi, size=3)
    bulk = np.stack([np.sin(k * x[:, (d + 1) % 3] + phase[d]) for d in range(3)], axis=1)
    v = vscale * (bulk + 0.3 * g.normal(size=(n, 3)))
    return x, v


def smooth_potential(seed: int, nm: int, n_modes: int = 12, amp: float = 1.0) -> np.ndarray:
    """A random periodic FP32 field [z,y,x] made of a few low-order Fourier modes."""
    g = rng(seed)
    i = np.arange(nm, dtype=np.float64)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    out = np.zeros((nm, nm, nm))
    for _ in range(n_modes):
        kv = g.integers(-3, 4, size=3)
        ph = g.uniform(0, 2 * np.pi)
        a = g.normal()
        out += a * np.cos(2 * np.pi * (kv[0] * x + kv[1] * y + kv[2] * z) / nm + ph)
    return (amp * out).astype(np.float32)


def random_field(seed: int, nm: int) -> np.ndarray:
    """Gaussian white noise [z,y,x] in FP32 (an arbitrary density for solver parity)."""
    return rng(seed).normal(size=(nm, nm, nm)).astype(np.float32)


def poisson_arrivals(seed: int, rate: float, n_jobs: int):
    """Exponential inter-arrival gaps (seconds) of a Poisson stream."""
    return np.cumsum(rng(seed).exponential(1.0 / rate, size=n_jobs))
