"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module holds none of the lattice Boltzmann method's arithmetic: it only
produces initial macroscopic fields, random numbers and network weights, all
in float64 on the host (the network weights are rounded once to float32).
Both the product path and the oracle turn these into populations themselves.

Workloads (the paper's datasets are not available; these analytic or seeded
fields stand in for them with the paper's shapes):

* ``tgv3d``: the three-dimensional Taylor-Green vortex of Sec. "Three-
  dimensional Taylor-Green Vortex" on [0, 2 pi)^3 with nodes at x_j = 2 pi j/N.
  The printed pressure is garbled; the standard one is used:
  p = rho0 u0^2 / 16 (cos 2x + cos 2y)(cos 2z + 2), rho = 1 + p / cs^2.
* ``tgv3d_octant``: the same vortex on the reduced domain of Appendix A,
  [0, pi/2]^3 with nodes half a spacing from the faces.
* ``tgv2d``: the two-dimensional Taylor-Green vortex of Sec. "Convergence",
  extruded along z without gradient, with its analytic velocity gradient.
  The printed pressure has the sign of the (sin x cos y, -cos x sin y) form
  of the vortex while the printed velocity is the (cos x sin y, -sin x cos y)
  form; the pressure that solves the Euler balance for the printed velocity
  is used: p = -rho0 u0^2/4 (cos 2x + cos 2y).
* ``turbulence``: a random-phase solenoidal field with
  E(k) ~ k^4 exp(-2 (k/k0)^2), scaled to a given rms velocity.
* ``mlp_params``: N(0, std) weights and biases drawn in the order W1, b1, W2,
  b2, ..., stored [in, out] row-major.
"""
import math

import numpy as np

CS2 = 1.0 / 3.0


def grid(n, offset=0.0):
    """Node coordinates x_j = 2 pi (j + offset) / n of a periodic box of edge 2 pi."""
    return 2.0 * np.pi * (np.arange(n) + offset) / n


def viscosity(n, u0, re):
    """Lattice viscosity for Reynolds number re = u0 L / nu with L = n / (2 pi)
    lattice units per unit length, and the BGK relaxation time tau = nu/cs^2 + 1/2."""
    nu = u0 * (n / (2.0 * np.pi)) / re
    return nu, nu / CS2 + 0.5


def tgv3d(n, u0, rho0=1.0, offset=0.0):
    """(rho, u) of the 3-D Taylor-Green vortex, shapes (n,n,n) and (3,n,n,n),
    index order [z, y, x]; nodes at 2 pi (j + offset) / n."""
    x = grid(n, offset)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.stack([u0 * np.sin(X) * np.cos(Y) * np.cos(Z),
                  -u0 * np.cos(X) * np.sin(Y) * np.cos(Z),
                  np.zeros_like(X)])
    p = rho0 * u0 * u0 / 16.0 * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    return rho0 + p / CS2, u


def tgv3d_octant(n, u0, rho0=1.0):
    """(rho, u) of the 3-D Taylor-Green vortex on the reduced domain of
    Appendix A ("Reduced Taylor-Green vortex"): the cube [0, pi/2]^3 with n
    nodes per edge, half a spacing from its faces, x_j = (j + 1/2) pi / (2 n).
    These are the first n nodes per axis of the 4n-node box with
    ``offset=0.5``; the spacing, and so the lattice viscosity of a Reynolds
    number, is that of the 4n box."""
    rho, u = tgv3d(4 * n, u0, rho0, offset=0.5)
    return rho[:n, :n, :n].copy(), u[:, :n, :n, :n].copy()


def tgv2d(n, u0, rho0=1.0):
    """(rho, u, grad_u) of the 2-D Taylor-Green vortex extruded along z.

    u = (u0 cos x sin y, -u0 sin x cos y, 0), p = -rho0 u0^2/4 (cos 2x + cos 2y).
    grad_u[a, b] = d u_b / d x_a in lattice units (one lattice spacing is
    2 pi / n)."""
    x = grid(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.stack([u0 * np.cos(X) * np.sin(Y), -u0 * np.sin(X) * np.cos(Y), np.zeros_like(X)])
    p = -rho0 * u0 * u0 / 4.0 * (np.cos(2 * X) + np.cos(2 * Y))
    s = 2.0 * np.pi / n
    g = np.zeros((3, 3) + X.shape)
    g[0, 0] = -u0 * np.sin(X) * np.sin(Y) * s
    g[1, 0] = u0 * np.cos(X) * np.cos(Y) * s
    g[0, 1] = -u0 * np.cos(X) * np.cos(Y) * s
    g[1, 1] = u0 * np.sin(X) * np.sin(Y) * s
    return rho0 + p / CS2, u, g


def turbulence(n, seed, k0=4.0, urms=0.05):
    """(rho, u): random-phase solenoidal velocity with model spectrum
    E(k) ~ k^4 exp(-2 (k/k0)^2), rms velocity ``urms`` per component, rho = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k1 = np.rint(np.fft.fftfreq(n, 1.0 / n))
    KZ, KY, KX = np.meshgrid(k1, k1, k1, indexing="ij")
    K = np.stack([KX, KY, KZ])
    kk = np.sqrt((K * K).sum(axis=0))
    amp = np.zeros_like(kk)
    nz = kk > 0
    # Shell energy E(k) spread over the 4 pi k^2 modes of the shell.
    amp[nz] = np.sqrt(kk[nz] ** 4 * np.exp(-2.0 * (kk[nz] / k0) ** 2) / (4.0 * np.pi * kk[nz] ** 2))
    noise = rng.standard_normal((3, n, n, n)) + 1j * rng.standard_normal((3, n, n, n))
    uh = noise * amp
    # Project onto divergence-free fields: uh -= k (k.uh) / |k|^2.
    kdot = (K * uh).sum(axis=0)
    uh[:, nz] -= K[:, nz] * kdot[nz] / (kk[nz] ** 2)
    u = np.real(np.fft.ifftn(uh, axes=(1, 2, 3)))
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    u *= urms / np.sqrt((u * u).mean())
    return np.ones((n, n, n)), u


def random_velocity(shape, seed, amp=0.05):
    """Uniform random velocity field in [-amp, amp]^3 and density in
    [0.95, 1.05], for parity tests far from any smooth flow."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = 1.0 + 0.05 * (2.0 * rng.random(shape) - 1.0)
    u = amp * (2.0 * rng.random((3,) + tuple(shape)) - 1.0)
    return rho, u


def random_populations(shape, seed, lo=0.5, hi=1.5):
    """Positive populations f_i(x) = r / 27 with r uniform in [lo, hi): a
    state far from equilibrium, used to exercise every moment."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (lo + (hi - lo) * rng.random((27,) + tuple(shape))) / 27.0


def mlp_params(width, seed, depth=2, std=0.1, n_in=27, n_out=4):
    """Flat float32-rounded parameter vector (returned as float64) for an MLP
    n_in -> width^depth -> n_out, all weights and biases N(0, std), drawn in
    the order W1, b1, W2, b2, ..., each W stored [in, out] row-major."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [n_in] + [width] * depth + [n_out]
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append(rng.normal(0.0, std, size=a * b))
        parts.append(rng.normal(0.0, std, size=b))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def n_params(width, depth=2, n_in=27, n_out=4):
    sizes = [n_in] + [width] * depth + [n_out]
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def alvelius_modes(kmax=2.0, kmin=0.0):
    """Integer wavevectors with kmin <= |k| <= kmax and k != 0, shape (n, 3) as
    (kx, ky, kz)."""
    r = int(math.floor(kmax))
    ks = [(kx, ky, kz) for kz in range(-r, r + 1) for ky in range(-r, r + 1) for kx in range(-r, r + 1)
          if 0 < kx * kx + ky * ky + kz * kz <= kmax * kmax and kx * kx + ky * ky + kz * kz >= kmin * kmin]
    return np.array(ks, dtype=np.int64)


def forcing_half_modes(kmax=2.0, kmin=0.0):
    """One wavevector of each +-k pair of ``alvelius_modes`` (the one whose
    first nonzero component, in the order z, y, x, is positive)."""
    ks = alvelius_modes(kmax, kmin)
    keep = [(kz > 0) or (kz == 0 and ky > 0) or (kz == 0 and ky == 0 and kx > 0) for kx, ky, kz in ks]
    return ks[np.array(keep)]


def uniform_draws(n_steps, n_modes, seed):
    """Uniform numbers in [0, 1), shape (n_steps, n_modes, 3): the random
    angles (phi, psi, theta1) of the spectral forcing, scaled to [0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((n_steps, n_modes, 3))
