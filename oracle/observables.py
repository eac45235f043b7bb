"""Observables of a lattice state, in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

* Global sums of mass and momentum (Sec. II.A, macroscopic moments) and the
  incompressible kinetic energy k = 1/2 <|u|^2> (Sec. on training with
  dissipation rates uses k and -dk/dt).
* The energy spectrum E(k) of the loss in Sec. "Learning Task".  The paper
  prints neither normalisation nor binning.  Reading: u_hat = DFT(u)/N^3 over
  integer wavevectors in [-N/2, N/2)^3 and E(k) = 1/2 sum of |u_hat|^2 over
  the shell round(|k|) = k, so that sum_k E(k) = 1/2 <|u|^2> (Parseval).
"""
import numpy as np

from . import collision


def global_sums(f):
    """(mass, j_x, j_y, j_z, 1/2 sum |u|^2) over all nodes."""
    rho, u = collision.macroscopic(f)
    j = rho * u
    return np.array([rho.sum(), j[0].sum(), j[1].sum(), j[2].sum(),
                     0.5 * (u * u).sum()])


def kinetic_energy(f):
    """k = 1/2 <|u|^2>, u = j / rho."""
    _, u = collision.macroscopic(f)
    return 0.5 * (u * u).sum(axis=0).mean()


def n_bins(n):
    """Number of shells round(|k|) = 0, 1, ... for a cubic grid of edge n."""
    return int(np.floor(np.sqrt(3.0) * (n // 2) + 0.5)) + 1


def wavenumbers(n):
    """Integer wavenumbers of DFT index 0..n-1, mapped into [-n/2, n/2)."""
    return np.rint(np.fft.fftfreq(n, 1.0 / n)).astype(np.int64)


def shell_index(n):
    """round(|k|) for every DFT index (kz, ky, kx) of a cubic grid."""
    k = wavenumbers(n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    return np.rint(np.sqrt(kx * kx + ky * ky + kz * kz)).astype(np.int64)


def spectrum_from_velocity(u):
    """E(k) of a velocity field u (3, n, n, n) via numpy's FFT."""
    n = u.shape[1]
    uh = np.fft.fftn(u, axes=(1, 2, 3)) / n ** 3
    e = 0.5 * (np.abs(uh) ** 2).sum(axis=0)
    return np.bincount(shell_index(n).ravel(), weights=e.ravel(), minlength=n_bins(n))


def spectrum_naive(u):
    """Same as ``spectrum_from_velocity`` by the DFT sum written out (small n)."""
    n = u.shape[1]
    x = np.arange(n)
    k = wavenumbers(n)
    E = np.zeros(n_bins(n))
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    for kz in k:
        for ky in k:
            for kx in k:
                phase = np.exp(-2j * np.pi * (kx * xx + ky * y + kz * z) / n)
                uh = (u * phase).sum(axis=(1, 2, 3)) / n ** 3
                b = int(np.rint(np.sqrt(kx * kx + ky * ky + kz * kz)))
                E[b] += 0.5 * float((np.abs(uh) ** 2).sum())
    return E


def spectrum(f):
    """E(k) of a lattice state (u = j / rho)."""
    _, u = collision.macroscopic(f)
    return spectrum_from_velocity(u)
