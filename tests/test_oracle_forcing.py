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


def test_phase_rule_matches_the_printed_tangent_and_decorrelates():
    """The velocity-dependent theta1: tan theta1 equals the printed ratio,
    and every forced mode's force is uncorrelated with the velocity there,
    so the force does no work on the field: sum_x F . u = 0."""
    rng = np.random.Generator(np.random.PCG64(71))
    n = 8
    u = 0.05 * rng.standard_normal((3, n, n, n))
    ks = inputs.forcing_half_modes(2.0)
    draw = rng.random((len(ks), 3))
    fh = forcing.coefficients_state(ks, draw, 1e-3, 1.5, 1.0, u)
    uh = forcing.velocity_modes(ks, u)
    for mi, k in enumerate(ks):
        assert abs(np.real(fh[mi] @ np.conj(uh[mi]))) < 1e-17
        e1, e2 = forcing.basis(k)
        xi1, xi2 = uh[mi] @ e1, uh[mi] @ e2
        phi, psi = np.pi * draw[mi, 0], 2 * np.pi * draw[mi, 1]
        ga, gb = np.sin(2 * phi), np.cos(2 * phi)
        num = ga * xi1.real + gb * (np.sin(psi) * xi2.imag + np.cos(psi) * xi2.real)
        den = -ga * xi1.imag + gb * (np.sin(psi) * xi2.real - np.cos(psi) * xi2.imag)
        assert np.isclose(np.tan(forcing.phase_rule(ga, gb, psi, xi1, xi2)), num / den, rtol=1e-10)
    F = forcing.field(ks, fh, (n, n, n))
    assert abs((F * u).sum()) < 1e-14 * np.abs(F).sum() * np.abs(u).max()
    # A random theta1 (the training forcing) does work on the same field.
    F0 = forcing.field(ks, forcing.coefficients(ks, draw[None], 1e-3, 1.5, 1.0)[0], (n, n, n))
    assert abs((F0 * u).sum()) > 1e-6 * np.abs(F0).sum() * np.abs(u).max()


def test_velocity_modes_match_the_fft():
    rng = np.random.Generator(np.random.PCG64(72))
    u = rng.standard_normal((3, 6, 5, 4))
    ks = np.array([[1, 0, 0], [0, 2, 1], [1, -1, 2]])
    uh = forcing.velocity_modes(ks, u)
    U = np.fft.fftn(u, axes=(1, 2, 3)) / (6 * 5 * 4)
    for mi, (kx, ky, kz) in enumerate(ks):
        assert np.allclose(uh[mi], U[:, kz % 6, ky % 5, kx % 4], atol=1e-15)


def test_field_vjp_is_the_transpose_of_field():
    """<field(d), g> = Re d . Re field_vjp(g) + Im d . Im field_vjp(g) for any
    coefficients d and weights g on a non-cubic grid."""
    ks = inputs.forcing_half_modes(2.0)[:6]
    rng = np.random.Generator(np.random.PCG64(81))
    shape = (5, 6, 7)
    d = rng.standard_normal((len(ks), 3)) + 1j * rng.standard_normal((len(ks), 3))
    g = rng.standard_normal((3,) + shape)
    lhs = (forcing.field(ks, d, shape) * g).sum()
    v = forcing.field_vjp(ks, g)
    rhs = (d.real * v.real).sum() + (d.imag * v.imag).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_phase_rule_vjp_matches_finite_differences():
    """Reverse mode of the velocity-dependent coefficients against central
    differences of ``coefficients_state`` along random velocity directions."""
    n = 6
    ks, draws = _forcing(1, seed=82)
    _, u = inputs.turbulence(n, seed=83, k0=2.0, urms=0.05)
    rng = np.random.Generator(np.random.PCG64(84))
    w = rng.standard_normal((len(ks), 3)) + 1j * rng.standard_normal((len(ks), 3))

    def loss(v):
        fh = forcing.coefficients_state(ks, draws[0], 1e-4, KF, CW, v)
        return (fh.real * w.real).sum() + (fh.imag * w.imag).sum()
    du = forcing.coefficients_state_vjp(ks, draws[0], 1e-4, KF, CW, u, w)
    h = 1e-7
    for _ in range(3):
        d = rng.standard_normal(u.shape) * 0.01
        fd = (loss(u + h * d) - loss(u - h * d)) / (2 * h)
        an = (du * d).sum()
        assert abs(fd - an) < 1e-6 * abs(an), (fd, an)
