"""Alvelius spectral forcing (Sec. "Training Data - Forced Isotropic
Turbulence"), in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

For a wavevector k with |k| = kk the force coefficient is
    F_hat(k) = A_ran e1(k) + B_ran e2(k),
    A_ran = (F(kk) / (2 pi kk^2))^(1/2) exp(i theta1) g_A(phi),
    B_ran = (F(kk) / (2 pi kk^2))^(1/2) exp(i theta2) g_B(phi),
    g_A = sin 2 phi, g_B = cos 2 phi, theta2 = theta1 + psi,
    F(kk) = A exp(-(kk - k_f)^2 / c),
with phi uniform in [0, pi), psi and theta1 uniform in [0, 2 pi).  The
amplitude A follows from the power input P over the time step dt (the
equation for A in the same section):
    A = (P / dt) / int_{k_a}^{k_b} exp(-(k - k_f)^2 / c) dk
(``amplitude_from_power``); the functions below also take A directly.

Readings: the printed e1 = (k_x k_y, -k_x k_y, 0)/sqrt(k_x^2 + k_y^2) is not
normal to k; the unit vector normal to k in the x-y plane,
e1 = (k_y, -k_x, 0)/sqrt(k_x^2 + k_y^2), is used, with e2 as printed; for
k_x = k_y = 0, e1 = (1, 0, 0) and e2 = (0, 1, 0).  theta1 is drawn from the
random numbers like phi and psi, so that the force is a known function of
time; ``coefficients_state`` is the velocity-dependent rule itself, and
``coefficients_state_vjp`` its reverse mode.  The force field is real: one
wavevector of each +-k pair carries F_hat and
F(x) = sum 2 Re(F_hat(k) exp(i k.x)), x in [0, 2 pi)^3.  F is the force per
unit mass: a step of length dt changes the velocity by F dt (the lattice's
own step has dt = 1).  k_a and k_b are the edges of the forced band of
wavenumbers, the integral's limits.
"""
import math

import numpy as np


def basis(k):
    """(e1, e2) for an integer wavevector k = (kx, ky, kz)."""
    kx, ky, kz = (float(v) for v in k)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    kp = np.sqrt(kx * kx + ky * ky)
    if kp == 0.0:
        return np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    e1 = np.array([ky, -kx, 0.0]) / kp
    e2 = np.array([kx * kz / kk, ky * kz / kk, -kp * kp / kk]) / kp
    return e1, e2


def spectrum(kk, amplitude, kf, c):
    """Force density F(k) = A exp(-(k - k_f)^2 / c), the Gaussian of the
    section's equation for F(k), at wavenumber magnitude kk."""
    return amplitude * np.exp(-(np.asarray(kk, dtype=np.float64) - kf) ** 2 / c)


def amplitude_from_power(power, dt, ka, kb, kf, c):
    """Amplitude A of F(k) for a power input P over a time step dt: the
    section's equation A = (P / dt) / int_{k_a}^{k_b} exp(-(k - k_f)^2 / c) dk,
    with the Gaussian's integral in closed form,
    sqrt(pi c) / 2 (erf((k_b - k_f) / sqrt c) - erf((k_a - k_f) / sqrt c))."""
    sc = math.sqrt(c)
    integral = 0.5 * math.sqrt(math.pi * c) * (math.erf((kb - kf) / sc) - math.erf((ka - kf) / sc))
    return (power / dt) / integral


def random_amplitudes(k, amplitude, kf, c, phi, psi, theta1):
    """(A_ran, B_ran) of the wavevector k for arrays of the angles phi, psi
    and theta1: (F(|k|) / (2 pi |k|^2))^(1/2) exp(i theta1) g_A(phi) and the
    same with theta2 = theta1 + psi and g_B(phi)."""
    kk = np.sqrt(float((np.asarray(k) ** 2).sum()))
    mag = np.sqrt(spectrum(kk, amplitude, kf, c) / (2.0 * np.pi * kk * kk))
    a = mag * np.exp(1j * theta1) * np.sin(2.0 * phi)
    b = mag * np.exp(1j * (theta1 + psi)) * np.cos(2.0 * phi)
    return a, b


def coefficients(ks, draws, amplitude, kf, c):
    """F_hat for every step and mode: ks (n_modes, 3) integers, draws
    (n_steps, n_modes, 3) uniform in [0, 1) as (phi, psi, theta1) / range.
    Returns complex (n_steps, n_modes, 3)."""
    ks = np.asarray(ks)
    draws = np.asarray(draws, dtype=np.float64)
    out = np.zeros(draws.shape[:2] + (3,), dtype=np.complex128)
    for mi, k in enumerate(ks):
        e1, e2 = basis(k)
        A, B = random_amplitudes(k, amplitude, kf, c, np.pi * draws[:, mi, 0], 2.0 * np.pi * draws[:, mi, 1],
                                 2.0 * np.pi * draws[:, mi, 2])
        out[:, mi, :] = A[:, None] * e1[None, :] + B[:, None] * e2[None, :]
    return out


def velocity_modes(ks, u):
    """u_hat(k) = N^-1 sum_x u(x) exp(-i k.x) at the given integer
    wavevectors, for a velocity field u (3, nz, ny, nx) on [0, 2 pi)^3
    (the coefficient of exp(i k.x) in u).  Returns complex (n_modes, 3)."""
    _, nz, ny, nx = u.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((len(ks), 3), dtype=np.complex128)
    for mi, k in enumerate(np.asarray(ks)):
        e = np.exp(-2j * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz))
        for a in range(3):
            out[mi, a] = (u[a] * e).sum() / u[a].size
    return out


def phase_rule(g_a, g_b, psi, xi1, xi2):
    """theta1 of Alvelius' rule (Sec. "Training Data - Forced Isotropic
    Turbulence", the tangent equation): the phase that makes the force of a
    mode uncorrelated with the velocity there, Re(F_hat . conj(u_hat)) = 0.
    With Z = g_A conj(xi1) + g_B exp(i psi) conj(xi2) that correlation is
    |A| Re(exp(i theta1) Z), zero for tan theta1 = Re Z / Im Z, which is the
    printed ratio (the stray factor e in front of tan is dropped).  Of the
    two solutions theta1 and theta1 + pi, atan2(Re Z, Im Z) is taken: it
    keeps F_hat continuous in u_hat (the other choice of branch flips the
    force's sign where Im Z changes sign)."""
    Z = g_a * np.conj(xi1) + g_b * np.exp(1j * psi) * np.conj(xi2)
    return np.arctan2(Z.real, Z.imag)


def coefficients_state(ks, draw, amplitude, kf, c, u):
    """F_hat of one step with the velocity-dependent theta1: draw (n_modes,
    3) as in ``coefficients`` (the theta1 column unused), u the velocity field
    the force acts on.  Returns complex (n_modes, 3)."""
    ks = np.asarray(ks)
    uh = velocity_modes(ks, u)
    out = np.zeros((len(ks), 3), dtype=np.complex128)
    for mi, k in enumerate(ks):
        e1, e2 = basis(k)
        phi, psi = np.pi * draw[mi, 0], 2.0 * np.pi * draw[mi, 1]
        ga, gb = np.sin(2.0 * phi), np.cos(2.0 * phi)
        th1 = phase_rule(ga, gb, psi, uh[mi] @ e1, uh[mi] @ e2)
        A, B = random_amplitudes(k, amplitude, kf, c, phi, psi, th1)
        out[mi] = A * e1 + B * e2
    return out


def coefficients_state_vjp(ks, draw, amplitude, kf, c, u, dfhat):
    """Reverse mode of ``coefficients_state``: dL/du (3, nz, ny, nx) for
    dfhat = dL/d Re F_hat + i dL/d Im F_hat (complex (n_modes, 3)).

    Per mode, backwards through the definitions above: F_hat is |A| e^{i
    theta1} (g_A e1 + g_B e^{i psi} e2), so dF_hat/d theta1 = i F_hat;
    theta1 = atan2(Re Z, Im Z) has gradient (Im Z, -Re Z) / |Z|^2 in (Re Z,
    Im Z) (taken as zero where Z = 0, where theta1 is not differentiable);
    Z = g_A conj(xi1) + g_B e^{i psi} conj(xi2) and xi_i = u_hat . e_i are
    real-linear, and u_hat = N^-1 sum_x u(x) e^{-i k.x}."""
    ks = np.asarray(ks)
    _, nz, ny, nx = u.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    uh = velocity_modes(ks, u)
    du = np.zeros(u.shape)
    for mi, k in enumerate(ks):
        e1, e2 = basis(k)
        phi, psi = np.pi * draw[mi, 0], 2.0 * np.pi * draw[mi, 1]
        ga, gb = np.sin(2.0 * phi), np.cos(2.0 * phi)
        xi1, xi2 = uh[mi] @ e1, uh[mi] @ e2
        Z = ga * np.conj(xi1) + gb * np.exp(1j * psi) * np.conj(xi2)
        th1 = np.arctan2(Z.real, Z.imag)
        A, B = random_amplitudes(k, amplitude, kf, c, phi, psi, th1)
        fh = A * e1 + B * e2
        d_th1 = float(np.sum(dfhat[mi].real * (1j * fh).real + dfhat[mi].imag * (1j * fh).imag))
        z2 = Z.real ** 2 + Z.imag ** 2
        if z2 == 0.0:
            continue
        dzr, dzi = d_th1 * Z.imag / z2, -d_th1 * Z.real / z2
        # Z.real = ga xi1.re + gb (cos psi xi2.re + sin psi xi2.im)
        # Z.imag = -ga xi1.im + gb (sin psi xi2.re - cos psi xi2.im)
        cp, sp = np.cos(psi), np.sin(psi)
        d1r, d1i = ga * dzr, -ga * dzi
        d2r, d2i = gb * (cp * dzr + sp * dzi), gb * (sp * dzr - cp * dzi)
        dur, dui = d1r * e1 + d2r * e2, d1i * e1 + d2i * e2
        # u_hat.re = N^-1 sum u cos(k.x), u_hat.im = -N^-1 sum u sin(k.x)
        th = 2.0 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz)
        cs, sn = np.cos(th), np.sin(th)
        for a in range(3):
            du[a] += (dur[a] * cs - dui[a] * sn) / cs.size
    return du


def field_vjp(ks, gF):
    """Transpose of ``field``: for gF = dL/dF (3, nz, ny, nx), the complex
    (n_modes, 3) array dL/d Re F_hat + i dL/d Im F_hat.  With F_a(x) =
    2 (Re F_hat_a cos(k.x) - Im F_hat_a sin(k.x)) that is
    2 sum_x gF_a(x) (cos(k.x) - i sin(k.x))."""
    _, nz, ny, nx = gF.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((len(ks), 3), dtype=np.complex128)
    for mi, k in enumerate(np.asarray(ks)):
        th = 2.0 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz)
        cs, sn = np.cos(th), np.sin(th)
        for a in range(3):
            out[mi, a] = 2.0 * (gF[a] * cs).sum() - 2.0j * (gF[a] * sn).sum()
    return out


def field(ks, fhat, shape):
    """Real force field (3, nz, ny, nx) of one step from its coefficients."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    F = np.zeros((3,) + tuple(shape))
    for k, fh in zip(np.asarray(ks), fhat):
        th = 2.0 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz)
        e = np.exp(1j * th)
        for a in range(3):
            F[a] += 2.0 * np.real(fh[a] * e)
    return F
