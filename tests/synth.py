"""Seeded synthetic inputs shared by the oracle and the HIP path in tests.

Only random numbers live here -- no arithmetic of the method.  Tests turn
these fields into populations with the oracle's initialiser and hand the same
population arrays to both sides.
"""
from __future__ import annotations

import numpy as np


def smooth_phase(nx, ny, nz, seed, n_modes=4, width=2.5):
    """A random smooth order-parameter-like field in [-1, 1]: tanh of a sum of
    periodic sinusoids, so that interfaces of width ~ ``width`` appear."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = np.zeros((nz, ny, nx))
    for _ in range(n_modes):
        kx, ky, kz = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        a = rng.uniform(0.5, 1.0)
        s += a * np.cos(2 * np.pi * kx * x / nx + ph[0]) * np.cos(2 * np.pi * ky * y / ny + ph[1]) \
            * np.cos(2 * np.pi * kz * z / nz + ph[2])
    s += rng.uniform(-0.2, 0.2)
    return np.tanh(s * width)


def smooth_velocity(nx, ny, nz, seed, amp=0.02):
    rng = np.random.default_rng(seed + 7)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((nz, ny, nx, 3))
    for c in range(3):
        k = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        u[..., c] = amp * np.sin(2 * np.pi * k[0] * x / nx + ph[0]) * np.sin(
            2 * np.pi * k[1] * y / ny + ph[1]) * np.cos(2 * np.pi * k[2] * z / nz + ph[2])
    return u.reshape(-1, 3)


def population_noise(n_nodes, seed, amp=1e-4):
    """Independent noise for the 2 x 27 populations of every node."""
    rng = np.random.default_rng(seed + 13)
    return amp * rng.standard_normal((2, 27, n_nodes))


def population_noise_planes(n_nodes, seed, amp=1e-4):
    """The values of population_noise, one (n_nodes,) plane at a time (red
    planes 0..26, then blue), for lattices where the whole array is large."""
    rng = np.random.default_rng(seed + 13)
    for _ in range(2 * 27):
        yield amp * rng.standard_normal(n_nodes)


def random_state_fields(prob, seed):
    """(rho_r, rho_b, u) of a random but physical state of ``prob``'s lattice."""
    phi = smooth_phase(prob.nx, prob.ny, prob.nz, seed).ravel()
    rng = np.random.default_rng(seed + 3)
    dens = 1.0 + 0.01 * rng.standard_normal(phi.shape)
    rho_r = prob.rho_r0 * (1 + phi) / 2 * dens
    rho_b = prob.rho_b0 * (1 - phi) / 2 * dens
    u = smooth_velocity(prob.nx, prob.ny, prob.nz, seed)
    return rho_r, rho_b, u
