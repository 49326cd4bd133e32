"""Seeded synthetic inputs for the D3Q19 binary-fluid lattice-Boltzmann step.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
only input recipes (random draws and analytic initial profiles) and parameter
sets; it contains none of the method's arithmetic (no moments, equilibria,
stencils, collision or streaming).

All arrays are float64 in C order with shape (nx, ny, nz); the last axis (z) is
contiguous in memory.  Random numbers come from a CPU ``torch.Generator`` with
an explicit seed and are drawn once, on the host, so that every consumer sees
identical bits.
"""
from __future__ import annotations

import math

import numpy as np
import torch

# Symmetric binary-fluid parameters used by every workload: free energy
# psi = A/2 phi^2 + B/4 phi^4 + kappa/2 |grad phi|^2, BGK relaxation times,
# the mobility parameter Gamma of the order-parameter equilibrium and the rest
# density.  Equilibrium bulk phases sit at phi = +-sqrt(-A/B) = +-1.
SPINODAL_PARAMS = dict(A=-0.00625, B=0.00625, kappa=0.004, gamma=0.5,
                       tau_f=1.0, tau_g=1.0, rho0=1.0)

# Default seeds: phi0 of the spinodal lattices, droplet noise, lamellar phase.
SEED_SPINODAL = 1234
SEED_DROPLET = 5678
SEED_LAMELLAR = 42


def _uniform(shape, seed: int) -> np.ndarray:
    """i.i.d. U[0, 1) float64 with a fixed CPU generator."""
    gen = torch.Generator(device="cpu")
    gen.manual_seed(int(seed))
    return torch.rand(tuple(shape), generator=gen, dtype=torch.float64).numpy()


def spinodal_phi0(shape, seed: int = SEED_SPINODAL, amp: float = 0.05) -> np.ndarray:
    """Initial order parameter for spinodal decomposition: i.i.d. U(-amp, amp)."""
    return amp * (2.0 * _uniform(shape, seed) - 1.0)


def interface_width(A: float, kappa: float) -> float:
    """Equilibrium interface width xi = sqrt(-2 kappa / A) of the tanh profile."""
    return math.sqrt(-2.0 * kappa / A)


def droplet_phi0(shape, radius: float, xi: float, noise: float = 1e-3,
                 seed: int = SEED_DROPLET) -> np.ndarray:
    """tanh droplet: phi = tanh((R - r)/xi) + U(-noise, noise).

    The centre is the lattice site (nx/2, ny/2, nz/2) with 0-based integer
    coordinates; phi is +1 inside and -1 outside.
    """
    nx, ny, nz = shape
    x = np.arange(nx, dtype=np.float64)[:, None, None] - nx // 2
    y = np.arange(ny, dtype=np.float64)[None, :, None] - ny // 2
    z = np.arange(nz, dtype=np.float64)[None, None, :] - nz // 2
    r = np.sqrt(x * x + y * y + z * z)
    phi = np.tanh((radius - r) / xi)
    if noise:
        phi = phi + noise * (2.0 * _uniform(shape, seed) - 1.0)
    return np.ascontiguousarray(phi)


def lamellar_target(shape, period: int, xi: float, seed: int = SEED_LAMELLAR) -> np.ndarray:
    """Lamellar target profile phi*(x) = tanh(d/xi), d = (P/2pi) sin(2pi (x+s)/P).

    The lamellae are normal to the first axis; the seed picks the integer phase
    s in [0, P).  d is the signed distance to the nearest interface to first
    order, so the profile has the equilibrium width near each interface.
    """
    nx, ny, nz = shape
    gen = torch.Generator(device="cpu")
    gen.manual_seed(int(seed))
    s = int(torch.randint(0, period, (1,), generator=gen).item())
    x = np.arange(nx, dtype=np.float64)
    d = (period / (2.0 * math.pi)) * np.sin(2.0 * math.pi * (x + s) / period)
    prof = np.tanh(d / xi)
    return np.ascontiguousarray(np.broadcast_to(prof[:, None, None], (nx, ny, nz)).copy())


def random_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Generic i.i.d. U(lo, hi) float64 field (test cotangents, perturbations)."""
    return lo + (hi - lo) * _uniform(shape, seed)
