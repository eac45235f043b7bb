"""Oracle pins of the spectral forcing (Sec. "Training Data - Forced
Isotropic Turbulence"): the force is solenoidal, its basis orthonormal, the
synthesised field real with the prescribed Fourier content; every mode
carries the force density F(|k|) / (2 pi |k|^2) of the section's equations
for A_ran and B_ran, split between e1 and e2 as tan 2 phi with the phase
offset psi; the amplitude A of F(k) follows from the power input, and the
force injects that power."""
import math

import numpy as np
import pytest
from scipy import integrate

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


# ---------------------------------------------------------------------------
# Amplitude, force density and power input.

def _split(ks, fh):
    """(A_ran, B_ran): the components of coefficients F_hat (..., n_modes, 3)
    along e1 and e2 of each mode."""
    a = np.zeros(fh.shape[:-1], dtype=np.complex128)
    b = np.zeros(fh.shape[:-1], dtype=np.complex128)
    for mi, k in enumerate(ks):
        e1, e2 = forcing.basis(k)
        a[..., mi] = fh[..., mi, :] @ e1
        b[..., mi] = fh[..., mi, :] @ e2
    return a, b


def _magnitude_error(ks, fh, amp, kf, c):
    """max |(|F_hat|^2 (2 pi |k|^2) / F(|k|)) - 1| over steps and modes: every
    mode carries the density F(|k|) / (2 pi |k|^2) whatever the angles (the
    basis is orthonormal and g_A^2 + g_B^2 = 1)."""
    kk = np.sqrt((np.asarray(ks, dtype=np.float64) ** 2).sum(axis=1))
    want = forcing.spectrum(kk, amp, kf, c) / (2.0 * np.pi * kk * kk)
    got = (np.abs(fh) ** 2).sum(axis=-1)
    return float(np.abs(got / want - 1.0).max())


def _ratio_phase_errors(ks, fh, phi, psi):
    """Largest deviations of |A_ran| / |B_ran| from |tan 2 phi| (relative)
    and of arg B_ran - arg A_ran from psi (mod 2 pi), over the modes where
    both are well away from zero."""
    a, b = _split(ks, fh)
    ok = (np.abs(np.sin(2 * phi)) > 0.05) & (np.abs(np.cos(2 * phi)) > 0.05)
    ratio = np.abs(np.abs(a[ok]) / np.abs(b[ok]) / np.abs(np.tan(2 * phi[ok])) - 1.0).max()
    # B_ran / A_ran = exp(i psi) cot 2 phi: its phase is psi, or psi + pi
    # where cot 2 phi < 0.
    q = b[ok] / a[ok] * np.sign(np.tan(2 * phi[ok]))
    dphase = np.angle(q * np.exp(-1j * psi[ok]))
    return float(ratio), float(np.abs(dphase).max())


def test_force_density_is_the_gaussian():
    """F(k_f) = A and F(k_f +- sqrt c) = A / e, F(k_f +- 2 sqrt c) = A e^-4."""
    amp, kf, c = 3e-4, 1.5, 0.7
    assert forcing.spectrum(kf, amp, kf, c) == amp
    for d, f in [(1.0, math.exp(-1.0)), (2.0, math.exp(-4.0))]:
        for sgn in (-1.0, 1.0):
            assert math.isclose(forcing.spectrum(kf + sgn * d * math.sqrt(c), amp, kf, c), amp * f, rel_tol=1e-14)


def test_unit_modes_carry_the_printed_density():
    """Worked values: with F(|k|) = 2 pi |k|^2 at the mode, |F_hat| = 1 for
    any angles (k = (1,0,0) at k_f = 1 with A = 2 pi; k = (0,2,0) at k_f = 2
    with A = 8 pi)."""
    rng = np.random.Generator(np.random.PCG64(5))
    for k, kf, amp in [((1, 0, 0), 1.0, 2 * np.pi), ((0, 2, 0), 2.0, 8 * np.pi), ((0, 0, 3), 3.0, 18 * np.pi)]:
        draws = rng.random((6, 1, 3))
        fh = forcing.coefficients(np.array([k]), draws, amp, kf, 1.0)
        np.testing.assert_allclose(np.abs(fh[:, 0, :]) ** 2 @ np.ones(3), 1.0, rtol=1e-14)


def test_every_mode_carries_the_force_density():
    """|F_hat(k)|^2 = F(|k|) / (2 pi |k|^2) for every mode and step, drawn
    phases and the velocity-dependent rule alike."""
    amp, kf, c = 2e-5, 1.5, 1.0
    ks = inputs.forcing_half_modes(2.5, 0.5)
    draws = inputs.uniform_draws(5, len(ks), seed=91)
    assert _magnitude_error(ks, forcing.coefficients(ks, draws, amp, kf, c), amp, kf, c) < 1e-13
    _, u = inputs.turbulence(8, seed=92, k0=2.0, urms=0.05)
    fh = forcing.coefficients_state(ks, draws[0], amp, kf, c, u)
    assert _magnitude_error(ks, fh, amp, kf, c) < 1e-13


def test_random_amplitudes_split_as_tan_two_phi_with_phase_offset_psi():
    """|A_ran| / |B_ran| = |tan 2 phi| and arg B_ran - arg A_ran = psi: the
    ratio of g_A = sin 2 phi to g_B = cos 2 phi and theta2 = theta1 + psi.
    With drawn phases arg A_ran is theta1 itself (up to the sign of g_A)."""
    amp, kf, c = 2e-5, 1.5, 1.0
    ks = inputs.forcing_half_modes(2.5, 0.5)
    draws = inputs.uniform_draws(6, len(ks), seed=93)
    phi, psi, th1 = np.pi * draws[..., 0], 2 * np.pi * draws[..., 1], 2 * np.pi * draws[..., 2]
    fh = forcing.coefficients(ks, draws, amp, kf, c)
    ratio, dphase = _ratio_phase_errors(ks, fh, phi, psi)
    assert ratio < 1e-12 and dphase < 1e-12
    a, _ = _split(ks, fh)
    assert np.abs(np.angle(a * np.sign(np.sin(2 * phi)) * np.exp(-1j * th1))).max() < 1e-12
    # The velocity-dependent rule keeps the split and the offset.
    _, u = inputs.turbulence(8, seed=94, k0=2.0, urms=0.05)
    fh = forcing.coefficients_state(ks, draws[0], amp, kf, c, u)
    ratio, dphase = _ratio_phase_errors(ks, fh, phi[0], psi[0])
    assert ratio < 1e-12 and dphase < 1e-12


def test_amplitude_from_power_matches_quadrature():
    """A = (P / dt) / int_{k_a}^{k_b} exp(-(k - k_f)^2 / c) dk: the closed
    form against numerical quadrature, and the whole-line limit sqrt(pi c)."""
    for p, dt, ka, kb, kf, c in [(0.1, 1.0, 0.5, 2.5, 1.5, 1.0), (2e-6, 0.5, 1.0, 2.0, 1.5, 0.3),
                                 (1e-3, 2.0, 3.0, 9.0, 4.0, 5.0)]:
        integral, _ = integrate.quad(lambda k: math.exp(-(k - kf) ** 2 / c), ka, kb, epsabs=0, epsrel=1e-13)
        assert math.isclose(forcing.amplitude_from_power(p, dt, ka, kb, kf, c), p / dt / integral, rel_tol=1e-12)
    assert math.isclose(forcing.amplitude_from_power(1.0, 1.0, -60.0, 60.0, 3.0, 2.0), 1.0 / math.sqrt(2.0 * math.pi),
                        rel_tol=1e-14)


POWER, DT, KA, KB, KFP, CP = 2e-6, 0.5, 0.5, 2.5, 1.5, 1.0


def _injected_power(ks, coef, u):
    """Mean kinetic-energy gain per unit time of one step of length DT under
    the force field of coefficients coef: <|u + F dt|^2 - |u|^2> / (2 dt)."""
    F = forcing.field(ks, coef, u.shape[1:])
    return float((((u + DT * F) ** 2).sum(axis=0) - (u ** 2).sum(axis=0)).mean() / (2.0 * DT))


def test_forcing_injects_the_power_input():
    """With A from the power input P, the force injects P: exactly per step
    under the velocity-dependent phase (the force does no work on u, so the
    gain is dt / 2 <|F|^2>, the same for every draw), and on average over
    draws with drawn phases, whose work on u has zero mean.  The modes are every integer wavevector of the
    band k_a <= |k| <= k_b; the only difference to P is that of the shell sum
    over those wavevectors to the equation's integral, 0.16 % for this band."""
    ks = inputs.forcing_half_modes(KB, KA)
    amp = forcing.amplitude_from_power(POWER, DT, KA, KB, KFP, CP)
    _, u = inputs.turbulence(8, seed=95, k0=2.0, urms=0.05)
    draws = inputs.uniform_draws(400, len(ks), seed=96)
    ruled = [_injected_power(ks, forcing.coefficients_state(ks, draws[t], amp, KFP, CP, u), u) for t in range(4)]
    assert np.ptp(ruled) < 1e-12 * POWER
    assert abs(ruled[0] / POWER - 1.0) < 3e-3, ruled[0] / POWER
    # Drawn phases: the work term <u . F> averages out over the draws (its
    # per-draw spread at this weaker velocity is ~4 % of P, 0.2 % over 400 draws).
    fh = forcing.coefficients(ks, draws, amp, KFP, CP)
    _, uw = inputs.turbulence(8, seed=95, k0=2.0, urms=2e-4)
    drawn = np.mean([_injected_power(ks, fh[t], uw) for t in range(len(draws))])
    assert abs(drawn / POWER - 1.0) < 0.015, drawn / POWER


def _slip_k_not_k2(k, amplitude, kf, c, phi, psi, theta1):
    kk = np.sqrt(float((np.asarray(k) ** 2).sum()))
    mag = np.sqrt(forcing.spectrum(kk, amplitude, kf, c) / (2.0 * np.pi * kk))
    return mag * np.exp(1j * theta1) * np.sin(2 * phi), mag * np.exp(1j * (theta1 + psi)) * np.cos(2 * phi)


def _slip_swapped_g(k, amplitude, kf, c, phi, psi, theta1):
    kk = np.sqrt(float((np.asarray(k) ** 2).sum()))
    mag = np.sqrt(forcing.spectrum(kk, amplitude, kf, c) / (2.0 * np.pi * kk * kk))
    return mag * np.exp(1j * theta1) * np.cos(2 * phi), mag * np.exp(1j * (theta1 + psi)) * np.sin(2 * phi)


def _slip_theta2(k, amplitude, kf, c, phi, psi, theta1):
    kk = np.sqrt(float((np.asarray(k) ** 2).sum()))
    mag = np.sqrt(forcing.spectrum(kk, amplitude, kf, c) / (2.0 * np.pi * kk * kk))
    return mag * np.exp(1j * theta1) * np.sin(2 * phi), mag * np.exp(1j * (theta1 - psi)) * np.cos(2 * phi)


@pytest.mark.parametrize("slip", ["k_not_k2", "swapped_g", "theta2", "power_times_dt", "no_2pi"])
def test_planted_forcing_mistakes_fail_the_pins(monkeypatch, slip):
    """Negative controls: a mistake planted in the oracle's forcing is caught
    by at least one of the pins above."""
    amp, kf, c = 2e-5, 1.5, 1.0
    ks = inputs.forcing_half_modes(2.5, 0.5)
    draws = inputs.uniform_draws(4, len(ks), seed=97)
    phi, psi = np.pi * draws[..., 0], 2 * np.pi * draws[..., 1]
    if slip == "k_not_k2":
        monkeypatch.setattr(forcing, "random_amplitudes", _slip_k_not_k2)
    elif slip == "swapped_g":
        monkeypatch.setattr(forcing, "random_amplitudes", _slip_swapped_g)
    elif slip == "theta2":
        monkeypatch.setattr(forcing, "random_amplitudes", _slip_theta2)
    elif slip == "power_times_dt":
        good = forcing.amplitude_from_power
        monkeypatch.setattr(forcing, "amplitude_from_power",
                            lambda p, dt, ka, kb, kf_, c_: good(p, dt, ka, kb, kf_, c_) * dt * dt)
    elif slip == "no_2pi":
        good_ra = forcing.random_amplitudes
        monkeypatch.setattr(forcing, "random_amplitudes",
                            lambda *a: tuple(v * math.sqrt(2 * math.pi) for v in good_ra(*a)))
    fh = forcing.coefficients(ks, draws, amp, kf, c)
    ratio, dphase = _ratio_phase_errors(ks, fh, phi, psi)
    caught = _magnitude_error(ks, fh, amp, kf, c) > 1e-6 or ratio > 1e-6 or dphase > 1e-6
    pks = inputs.forcing_half_modes(KB, KA)
    _, u = inputs.turbulence(8, seed=95, k0=2.0, urms=0.05)
    pa = forcing.amplitude_from_power(POWER, DT, KA, KB, KFP, CP)
    pd = inputs.uniform_draws(1, len(pks), seed=98)
    gain = _injected_power(pks, forcing.coefficients_state(pks, pd[0], pa, KFP, CP, u), u)
    caught = caught or abs(gain / POWER - 1.0) > 3e-3
    assert caught, slip
