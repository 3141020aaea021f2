"""Seeded synthetic workloads: lattice parameters and random inputs.

This module holds no arithmetic of the method.  It only fixes the workload
parameters (lattice sizes, relaxation times, noise temperature, mean velocity,
step counts, seeds) and draws seeded random arrays, so that the GPU library
and the oracle can be fed exactly the same inputs.

Relaxation-time vectors are indexed by moment a = 0..8 (0 density, 1-2
momentum, 3-4 shear stress, 5 bulk stress, 6-8 ghost modes); entries 0..2 are
ignored by the method because those moments are conserved.
"""
from __future__ import annotations

import numpy as np


def tau_vector(shear, bulk, ghost):
    return [1.0, 1.0, 1.0, float(shear), float(shear), float(bulk),
            float(ghost), float(ghost), float(ghost)]


# Workloads with the shapes of the paper's runs and of the benchmark suite of
# this library.  theta is the noise temperature (k_B T = 1/3 reproduces the
# paper's unit-mass variance exactly).
CONFIGS = {
    # 32^2, tau_shear = tau_bulk = 0.8, ghost 1, seed 1, 1e4 steps, sample /10
    "c1_32": dict(nx=32, ny=32, tau=tau_vector(0.8, 0.8, 1.0), theta=1e-4, rho0=1.0,
                  u0=(0.0, 0.0), seed=1, steps=10_000, sample_every=10),
    # 256^2, tau_shear 0.8, bulk 1, ghost 1, 1e5 steps, sample /10
    "c2_256": dict(nx=256, ny=256, tau=tau_vector(0.8, 1.0, 1.0), theta=1e-4, rho0=1.0,
                   u0=(0.0, 0.0), seed=2, steps=100_000, sample_every=10),
    # 4096^2, u0_x = 0.05, tau_shear 0.6, 2e4 steps, sample /10
    "c5_4096": dict(nx=4096, ny=4096, tau=tau_vector(0.6, 1.0, 1.0), theta=1e-4, rho0=1.0,
                    u0=(0.05, 0.0), seed=5, steps=20_000, sample_every=10),
    # the paper's own regime: V = 20^2, tau^a = 1 for all a
    "paper_20": dict(nx=20, ny=20, tau=tau_vector(1.0, 1.0, 1.0), theta=1e-4, rho0=1.0,
                     u0=(0.0, 0.0), seed=7, steps=200_000, sample_every=1),
}

# Galilean-invariance sweep: 16 realisations of 512^2 per mean velocity.
GI_VELOCITIES = (0.0, 0.025, 0.05, 0.1, 0.15, 0.2)


def gi_sweep_specs(n_per_velocity=16, side=512):
    specs = []
    for iu, u in enumerate(GI_VELOCITIES):
        for r in range(n_per_velocity):
            specs.append(dict(nx=side, ny=side, tau=tau_vector(0.8, 1.0, 1.0), theta=1e-4,
                              rho0=1.0, u0=(u, 0.0), stream_id=n_per_velocity * iu + r))
    return specs


def uneven_batch_specs(n=64, seed=4, lo=64, hi=1024):
    """64 lattices, sides log-uniform in [lo, hi], tau_shear U[0.55, 1.5],
    u0_x U[0, 0.1]; independent nx, ny."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        nx, ny = (int(round(np.exp(rng.uniform(np.log(lo), np.log(hi))))) for _ in range(2))
        ts = float(rng.uniform(0.55, 1.5))
        ux = float(rng.uniform(0.0, 0.1))
        specs.append(dict(nx=nx, ny=ny, tau=tau_vector(ts, 1.0, 1.0), theta=1e-4, rho0=1.0,
                          u0=(ux, 0.0), stream_id=i))
    return specs


def perturbed(base9, nx, ny, amp, seed):
    """base9[i] + amp * N(0,1) independently at every population and site:
    an arbitrary (non-equilibrium) state of shape (9, ny, nx)."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base9, dtype=np.float64).reshape(9, 1, 1)
    return base + amp * rng.standard_normal((9, ny, nx))
