"""Oracle pins of the spectral forcing (Sec. "Training Data - Forced
Isotropic Turbulence"): the force is solenoidal, its basis orthonormal, the
synthesised field real with the prescribed Fourier content."""
import numpy as np

from oracle import forcing
from paper_2412_08229_amd import inputs

AMP, KF, CW = 2e-6, 1.5, 1.0


def _forcing(n_steps, seed):
    ks = inputs.forcing_half_modes(2.0)
    return ks, inputs.uniform_draws(n_steps, len(ks), seed)


def test_forcing_is_solenoidal_and_real():
    """Oracle pins of the spectral force: k . F_hat = 0 and |e1| = |e2| = 1."""
    ks, draws = _forcing(2, seed=3)
    fh = forcing.coefficients(ks, draws, AMP, KF, CW)
    for k, c in zip(ks, fh[0]):
        assert abs(np.dot(k, c)) < 1e-18
        e1, e2 = forcing.basis(k)
        assert abs(np.linalg.norm(e1) - 1) < 1e-15 and abs(np.linalg.norm(e2) - 1) < 1e-15
        assert abs(np.dot(e1, e2)) < 1e-15 and abs(np.dot(e1, k)) < 1e-15 and abs(np.dot(e2, k)) < 1e-15




def test_half_modes_cover_all_pairs():
    ks = inputs.forcing_half_modes(2.0)
    full = {tuple(k) for k in inputs.alvelius_modes(2.0)}
    assert len(full) == 32 and len(ks) == 16
    assert {tuple(k) for k in ks} | {tuple(-k) for k in ks} == full


def test_field_has_the_prescribed_fourier_coefficients():
    n = 8
    ks, draws = _forcing(1, seed=4)
    fh = forcing.coefficients(ks, draws, AMP, KF, CW)[0]
    F = forcing.field(ks, fh, (n, n, n))
    Fh = np.fft.fftn(F, axes=(1, 2, 3)) / n ** 3
    for k, c in zip(ks, fh):
        np.testing.assert_allclose(Fh[:, k[2] % n, k[1] % n, k[0] % n], c, rtol=1e-12, atol=1e-18)
    assert abs(F.mean()) < 1e-20
