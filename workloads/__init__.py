"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and lays out initial fields; it holds
none of the method's arithmetic.  Everything is float64 numpy, generated with
numpy's PCG64 so a seed gives the same arrays on every machine.

Workloads (initial states of the paper's benchmarks):
* Taylor-Green vortex, Sec. 7.1 Eq. (tg-initial-conditions): on an L x L
  grid, x_j = 2 pi j / L, u_x = u0 cos(x) sin(y), u_y = -u0 cos(y) sin(x),
  with n and T constant (optionally a seeded Gaussian perturbation of n).
* Shock tube (Riemann problem), Sec. 8.2: a left and a right state at rest
  split by a plane x = x0.
* Population noise: xi_i(x) ~ U[-1, 1], multiplied in as f_i (1 + amp xi_i).
* A batch of independent lattices with sides, tau and zeta drawn from a seed.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def taylor_green_2d(nx: int, ny: int, u0: float, n0: float = 1.0, T0: float = 1.0,
                    density_sigma: float = 0.0, seed: int | None = None, phase=(0.0, 0.0)):
    """Return n (ny, nx), T (ny, nx), u (2, ny, nx) for the Taylor-Green vortex."""
    x = 2.0 * np.pi * np.arange(nx) / nx + phase[0]
    y = 2.0 * np.pi * np.arange(ny) / ny + phase[1]
    X, Y = np.meshgrid(x, y)                      # shape (ny, nx)
    u = np.stack([u0 * np.cos(X) * np.sin(Y), -u0 * np.cos(Y) * np.sin(X)])
    n = np.full((ny, nx), n0, dtype=np.float64)
    if density_sigma > 0.0:
        n = n + density_sigma * rng(seed).standard_normal((ny, nx))
    T = np.full((ny, nx), T0, dtype=np.float64)
    return n, T, u


def taylor_green_3d(nx: int, ny: int, nz: int, u0: float, n0: float = 1.0, T0: float = 1.0,
                    density_sigma: float = 0.0, seed: int | None = None):
    """Return n, T (nz, ny, nx) and u (3, nz, ny, nx) for the 3D Taylor-Green vortex
    u = u0 (sin x cos y cos z, -cos x sin y cos z, 0), with optional Gaussian density noise."""
    x = 2.0 * np.pi * np.arange(nx) / nx
    y = 2.0 * np.pi * np.arange(ny) / ny
    z = 2.0 * np.pi * np.arange(nz) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")     # shape (nz, ny, nx)
    u = np.stack([u0 * np.sin(X) * np.cos(Y) * np.cos(Z), -u0 * np.cos(X) * np.sin(Y) * np.cos(Z),
                  np.zeros_like(X)])
    n = np.full((nz, ny, nx), n0, dtype=np.float64)
    if density_sigma > 0.0:
        n = n + density_sigma * rng(seed).standard_normal((nz, ny, nx))
    T = np.full((nz, ny, nx), T0, dtype=np.float64)
    return n, T, u


def riemann_3d(nx: int, ny: int, nz: int, x0: int, nL: float, TL: float, nR: float, TR: float):
    """Return n, T (nz, ny, nx) and u (3, nz, ny, nx) = 0 for a shock tube split at x = x0."""
    n = np.where(np.arange(nx)[None, None, :] < x0, nL, nR) * np.ones((nz, ny, 1))
    T = np.where(np.arange(nx)[None, None, :] < x0, TL, TR) * np.ones((nz, ny, 1))
    u = np.zeros((3, nz, ny, nx))
    return n.astype(np.float64), T.astype(np.float64), u


def population_noise(Q: int, grid_shape, seed: int) -> np.ndarray:
    """xi ~ U[-1, 1] with shape (Q, *grid_shape)."""
    return rng(seed).uniform(-1.0, 1.0, size=(Q,) + tuple(grid_shape))


def batch_lattices(count: int, seed: int, side_range=(64, 512), tau_range=(0.6, 2.0),
                   zeta_range=(0.0, 5.0)):
    """Sides uniform in {lo..hi}, tau ~ U[tau_range], zeta ~ U[zeta_range]."""
    g = rng(seed)
    sides = g.integers(side_range[0], side_range[1] + 1, size=count)
    taus = g.uniform(*tau_range, size=count)
    zetas = g.uniform(*zeta_range, size=count)
    return sides, taus, zetas


def batch_specs(count: int, seed: int, **kw):
    """batch_lattices as a list of {extent: (side, side), tau, zeta} dicts."""
    sides, taus, zetas = batch_lattices(count, seed, **kw)
    return [{"extent": (int(s), int(s)), "tau": float(t), "zeta": float(z)} for s, t, z in zip(sides, taus, zetas)]


def random_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=tuple(shape))
