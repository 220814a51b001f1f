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


def sphere_blobs(nx, ny, nz, seed, n_blobs, r_min=0.8, r_max=4.0):
    """An order-parameter-like field (node order) of +-1 with values in
    [0.3, 1] inside n_blobs random spheres (some overlapping, some cut by the
    lattice faces) and in [-1, -0.3] outside: many connected components with
    no value near 0."""
    rng = np.random.default_rng(seed)
    inside = np.zeros((nz, ny, nx), bool)
    cs = rng.uniform([0, 0, 0], [nx, ny, nz], size=(n_blobs, 3))
    rs = rng.uniform(r_min, r_max, size=n_blobs)
    for c, r in zip(cs, rs):
        lo = np.maximum(np.floor(c - r).astype(int), 0)
        hi = np.minimum(np.ceil(c + r).astype(int) + 1, [nx, ny, nz])
        z, y, x = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]),
                              indexing="ij")
        inside[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 < r * r
    mag = rng.uniform(0.3, 1.0, size=inside.shape)
    return np.where(inside, mag, -mag).ravel()


def population_noise(n_nodes, seed, amp=1e-4, q=27):
    """Independent noise for the 2 x q populations of every node."""
    rng = np.random.default_rng(seed + 13)
    return amp * rng.standard_normal((2, q, n_nodes))


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


def separable_state_fields(prob, seed, amp_u=0.02):
    """(rho_r, rho_b, u) of a random physical state built from products of 1-D
    waves (float32, node order), cheap enough for lattices of 10^8 nodes:
    phi = tanh(2.5 (sum_k a_k X_k(x) Y_k(y) Z_k(z) + c)) with interfaces, a
    1 % density modulation, smooth velocities of magnitude <= amp_u."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    ax = [np.arange(n, dtype=np.float64) for n in (nx, ny, nz)]

    def wave(n_ax, k_max):
        k = rng.integers(1, k_max + 1)
        ph = rng.uniform(0, 2 * np.pi)
        return np.cos(2 * np.pi * k * ax[n_ax] / len(ax[n_ax]) + ph)

    s = np.full((nz, ny, nx), rng.uniform(-0.2, 0.2), np.float32)
    for _ in range(3):
        a = rng.uniform(0.5, 1.0)
        X, Y, Z = wave(0, 3), wave(1, 3), wave(2, 3)
        s += (a * Z[:, None, None] * Y[None, :, None] * X[None, None, :]).astype(np.float32)
    phi = np.tanh(2.5 * s).ravel()
    del s
    X, Y, Z = wave(0, 7), wave(1, 7), wave(2, 7)
    dens = (1.0 + 0.01 * (Z[:, None, None] * Y[None, :, None] * X[None, None, :])).astype(np.float32).ravel()
    rho_r = (prob.rho_r0 * 0.5 * (1.0 + phi) * dens).astype(np.float32)
    rho_b = (prob.rho_b0 * 0.5 * (1.0 - phi) * dens).astype(np.float32)
    del phi, dens
    u = np.empty((nz * ny * nx, 3), np.float32)
    for c in range(3):
        X, Y, Z = wave(0, 2), wave(1, 2), wave(2, 2)
        u[:, c] = (amp_u * Z[:, None, None] * Y[None, :, None] * X[None, None, :]).astype(np.float32).ravel()
    return rho_r, rho_b, u


def droplet_profile(n, R, W, center=None):
    """The order parameter of the static droplet of Sec. III on an n^3
    lattice, phi = -tanh(2 (r - R) / W) (node order, x fastest)."""
    c = (n - 1) / 2.0 if center is None else center
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2).ravel()
    return -np.tanh(2.0 * (r - R) / W)
