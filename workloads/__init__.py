"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the lattice Boltzmann method: only the
workload parameters and seeded random initial fields / replica tables.  Both
the HIP path and the CPU oracle consume what it returns.

Workloads (all periodic, lattice units, k_B = 1):
  c0  D2Q9 64x64, FP64, ideal mixture G = 0, rho0 = 1 per species, tau = 1,
      k_BT = 1e-4, uniform start, seed 1.
  c1  D2Q9 1024x1024, FP32, G = 0.5, tau = (0.8, 1.2), tau_d = 1, k_BT = 1e-5,
      rho = 1 + U(-0.01, 0.01) per species and site, seed 1.
  c2  D3Q19 256^3, FP32, G = 1.2, tau = 1, k_BT = 1e-5,
      rho = 1 + U(-0.01, 0.01), seed 1.
  c3  as c2 with 16-bit deviation storage (bf16 or f16).
  c4  512 D2Q9 replicas, L = round(32 * 8**U) (log-uniform in [32, 256]),
      seed 1 + r, k_BT log-uniform in [1e-6, 1e-4], G ~ U(0, 1), tau = 1,
      uniform rho = 1, FP32.
The paper's own workloads (Sec. VI) are synthetic as well: uniform or
perturbed initial densities on small periodic boxes.
"""
from __future__ import annotations

import numpy as np

CONFIGS = {
    "c0": dict(lattice="d2q9", nx=64, ny=64, nz=1, storage="f64", G=0.0, tau=(1.0, 1.0),
               tau_d=1.0, kT=1e-4, seed=1, init="uniform", steps=1000),
    "c1": dict(lattice="d2q9", nx=1024, ny=1024, nz=1, storage="f32", G=0.5, tau=(0.8, 1.2),
               tau_d=1.0, kT=1e-5, seed=1, init="perturbed", steps=10000),
    "c2": dict(lattice="d3q19", nx=256, ny=256, nz=256, storage="f32", G=1.2, tau=(1.0, 1.0),
               tau_d=1.0, kT=1e-5, seed=1, init="perturbed", steps=5000),
    "c3": dict(lattice="d3q19", nx=256, ny=256, nz=256, storage="bf16", G=1.2, tau=(1.0, 1.0),
               tau_d=1.0, kT=1e-5, seed=1, init="perturbed", steps=5000),
}


def initial_density(shape, kind: str = "uniform", seed: int = 1, rho0=(1.0, 1.0),
                    amplitude: float = 0.01):
    """(rho1, rho2) arrays of the given lattice shape (nz, ny, nx).

    kind "uniform": rho_sigma = rho0_sigma everywhere.
    kind "perturbed": rho_sigma = rho0_sigma * (1 + U(-amplitude, amplitude)),
    independently per species and site, from numpy's PCG64 seeded with `seed`.
    """
    shape = tuple(int(s) for s in shape)
    if kind == "uniform":
        return (np.full(shape, float(rho0[0])), np.full(shape, float(rho0[1])))
    if kind == "perturbed":
        rng = np.random.default_rng(seed)
        r1 = rho0[0] * (1.0 + rng.uniform(-amplitude, amplitude, size=shape))
        r2 = rho0[1] * (1.0 + rng.uniform(-amplitude, amplitude, size=shape))
        return r1, r2
    raise ValueError(kind)


def stripe_density(nx: int, ny: int, width: int, dense: float = 2.3, light: float = 0.06):
    """Flat liquid stripe (Sec. VI B): species 1 dense inside the central
    `width` columns, species 2 dense outside.  Shape (1, ny, nx)."""
    x = np.arange(nx)
    lo = (nx - width) // 2
    inside = (x >= lo) & (x < lo + width)
    r1 = np.where(inside, dense, light)
    r2 = np.where(inside, light, dense)
    return (np.broadcast_to(r1, (1, ny, nx)).copy(), np.broadcast_to(r2, (1, ny, nx)).copy())


def replica_table(n: int = 512, master_seed: int = 2024, lmin: int = 32, lmax: int = 256):
    """Per-replica parameters of the batched workload: list of dicts with
    L (square side, log-uniform in [lmin, lmax]), seed, kT (log-uniform in
    [1e-6, 1e-4]) and G (uniform in [0, 1))."""
    rng = np.random.default_rng(master_seed)
    U = rng.uniform(0.0, 1.0, size=n)
    L = np.rint(lmin * (lmax / lmin) ** U).astype(int)
    kT = 10.0 ** rng.uniform(-6.0, -4.0, size=n)
    G = rng.uniform(0.0, 1.0, size=n)
    return [dict(L=int(L[r]), seed=1 + r, kT=float(kT[r]), G=float(G[r]), tau=(1.0, 1.0),
                 tau_d=1.0) for r in range(n)]
