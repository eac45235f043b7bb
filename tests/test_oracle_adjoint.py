"""Pins of the oracle's hand-written reverse mode against central finite
differences of the (separately pinned) forward oracle, in float64."""
import numpy as np
import pytest

from oracle import adjoint, collision, forcing, observables, step
from paper_2412_08229_amd import inputs


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _layers(width=8, seed=0):
    return collision.unpack_params(inputs.mlp_params(width, seed), width)


def _perturb(layers, v, h):
    out, pos = [], 0
    for W, b in layers:
        dW = v[pos:pos + W.size].reshape(W.shape)
        pos += W.size
        db = v[pos:pos + b.size]
        pos += b.size
        out.append((W + h * dW, b + h * db))
    return out


def test_equilibrium_vjp_matches_finite_differences():
    rng = _rng(1)
    f = inputs.random_populations((5,), seed=2)
    v = rng.standard_normal((27, 5))
    d = rng.standard_normal((27, 5))
    rho = f.sum(0)
    j = adjoint._C.T @ f

    def feq(g):
        r, u = collision.macroscopic(g)
        return collision.equilibrium(r, u)
    h = 1e-6
    fd = ((feq(f + h * d) - feq(f - h * d)) / (2 * h) * v).sum()
    an = (adjoint.equilibrium_vjp(rho, j, v) * d).sum()
    assert abs(fd - an) < 1e-8 * max(1.0, abs(an))


@pytest.mark.parametrize("act", ["tanh", "relu"])
@pytest.mark.parametrize("forced", [False, True])
def test_collision_vjp_matches_finite_differences(act, forced):
    rng = _rng(3)
    f = inputs.random_populations((6,), seed=4, lo=0.8, hi=1.2)
    lam = rng.standard_normal((27, 6))
    layers = _layers(8, 5)
    force = 1e-3 * rng.standard_normal((3, 6)) if forced else None
    tau = 0.56

    def post(g, lay):
        out = collision.nco(g, tau, lay, act)
        if forced:
            out = out + collision.kupershtokh_source(g, force)
        return out
    g_f, g_p = adjoint.nco_collide_vjp(f, lam, tau, layers, act, force)
    # ReLU is piecewise linear: a pre-activation lies 7e-6 from its kink
    # here, so the step must stay below that.
    h, tol = (1e-6, 1e-7) if act == "tanh" else (1e-8, 1e-6)
    d = rng.standard_normal((27, 6))
    fd = ((post(f + h * d, layers) - post(f - h * d, layers)) / (2 * h) * lam).sum()
    assert abs(fd - (g_f * d).sum()) < tol * max(1.0, abs(fd))
    v = rng.standard_normal(collision.n_params(8))
    fd = ((post(f, _perturb(layers, v, h)) - post(f, _perturb(layers, v, -h))) / (2 * h) * lam).sum()
    an = adjoint.flatten(g_p) @ v
    assert abs(fd - an) < tol * max(1.0, abs(an))


def test_spectrum_vjp_matches_finite_differences():
    rng = _rng(6)
    n = 6
    rho, u = inputs.random_velocity((n, n, n), seed=7)
    f = collision.equilibrium(rho, u)
    dE = rng.standard_normal(observables.n_bins(n))
    d = 1e-3 * rng.standard_normal(f.shape)
    h = 1e-6
    fd = ((observables.spectrum(f + h * d) - observables.spectrum(f - h * d)) / (2 * h) * dE).sum()
    an = (adjoint.spectrum_vjp(f, dE) * d).sum()
    assert abs(fd - an) < 1e-8 * max(abs(an), 1e-12)


def test_unrolled_gradient_matches_finite_differences():
    """Loss on log E(k) after 4 forced NCO steps on 6^3: gradient with respect
    to the network parameters and to the initial populations."""
    n, width, tau, T = 6, 8, 0.55, 4
    rng = _rng(8)
    layers = _layers(width, 9)
    _, u = inputs.turbulence(n, seed=10, k0=2.0, urms=0.05)
    f0 = collision.equilibrium(np.ones((n, n, n)), u)
    Et = observables.spectrum(f0) * 0.8 + 1e-9
    forces = [1e-4 * rng.standard_normal((3, n, n, n)) for _ in range(T)]

    def loss_grad(x):
        L, dE = adjoint.log_spectrum_loss(observables.spectrum(x), Et, 1, 3)
        return L, adjoint.spectrum_vjp(x, dE)

    def loss(lay, g0):
        op = step.Operator("nco", tau, layers=lay, act="tanh")
        return loss_grad(step.run(g0, op, T, forces=lambda t: forces[t]))[0]
    L, gp, gf0 = adjoint.run_and_grad(f0, tau, layers, "tanh", T, loss_grad, forces=lambda t: forces[t])
    assert abs(L - loss(layers, f0)) < 1e-14
    h = 1e-6
    v = rng.standard_normal(collision.n_params(width))
    fd = (loss(_perturb(layers, v, h), f0) - loss(_perturb(layers, v, -h), f0)) / (2 * h)
    an = adjoint.flatten(gp) @ v
    assert abs(fd - an) < 1e-6 * max(abs(an), 1e-12), (fd, an)
    d = 1e-3 * rng.standard_normal(f0.shape)
    fd = (loss(layers, f0 + h * d) - loss(layers, f0 - h * d)) / (2 * h)
    an = (gf0 * d).sum()
    assert abs(fd - an) < 1e-6 * max(abs(an), 1e-12), (fd, an)


def test_adjoint_negative_control():
    """A wrong streaming transpose (pull instead of push) breaks the check."""
    n, width, tau, T = 4, 8, 0.55, 2
    layers = _layers(width, 11)
    f0 = inputs.random_populations((n, n, n), seed=12, lo=0.9, hi=1.1)
    w = _rng(13).standard_normal(f0.shape)

    def loss_grad(x):
        return float((w * x).sum()), w
    _, _, good = adjoint.run_and_grad(f0, tau, layers, "tanh", T, loss_grad)
    saved = step.unstream
    try:
        step.unstream = step.stream
        _, _, bad = adjoint.run_and_grad(f0, tau, layers, "tanh", T, loss_grad)
    finally:
        step.unstream = saved
    assert np.abs(good - bad).max() > 1e-3


def test_kinetic_energy_vjp_matches_finite_differences():
    n = 4
    rng = _rng(14)
    rho, u = inputs.random_velocity((n, n, n), seed=15, amp=0.1)
    f = collision.equilibrium(rho, u) + 1e-3 * rng.standard_normal((27, n, n, n))
    g = adjoint.kinetic_energy_vjp(f)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(f.shape)
        fd = (observables.kinetic_energy(f + h * d) - observables.kinetic_energy(f - h * d)) / (2 * h)
        assert abs(fd - (g * d).sum()) < 1e-8 * abs(fd), (fd, (g * d).sum())


def test_trajectory_loss_gradient_matches_finite_differences():
    """A loss on the kinetic energy of intermediate states (the dissipation
    training of Sec. "Learning Task"): L = sum_m a_m k(t_m) over the states
    t = 0, 2, 4 of a 4-step NCO run on 4^3, plus the final-state term 0."""
    n, width, tau, T, every = 4, 8, 0.55, 4, 2
    rng = _rng(16)
    layers = _layers(width, 17)
    rho, u = inputs.random_velocity((n, n, n), seed=18, amp=0.08)
    f0 = collision.equilibrium(rho, u)
    a = rng.standard_normal(T // every + 1)

    def loss(lay, g0):
        op = step.Operator("nco", tau, layers=lay, act="tanh")
        x, total = g0, a[0] * observables.kinetic_energy(g0)
        for t in range(1, T + 1):
            x = step.step(x, op)
            if t % every == 0:
                total += a[t // every] * observables.kinetic_energy(x)
        return total

    def traj(t, x):
        return a[t // every] * adjoint.kinetic_energy_vjp(x) if t % every == 0 else None
    _, gp, gf0 = adjoint.run_and_grad(f0, tau, layers, "tanh", T, lambda x: (0.0, np.zeros_like(x)),
                                      traj_grad=traj)
    h = 1e-6
    v = rng.standard_normal(collision.n_params(width))
    fd = (loss(_perturb(layers, v, h), f0) - loss(_perturb(layers, v, -h), f0)) / (2 * h)
    an = adjoint.flatten(gp) @ v
    assert abs(fd - an) < 1e-6 * max(abs(an), 1e-12), (fd, an)
    d = 1e-3 * rng.standard_normal(f0.shape)
    fd = (loss(layers, f0 + h * d) - loss(layers, f0 - h * d)) / (2 * h)
    an = (gf0 * d).sum()
    assert abs(fd - an) < 1e-6 * max(abs(an), 1e-12), (fd, an)


def test_collision_vjp_depth3_matches_finite_differences():
    """The reverse mode through a network with a third hidden layer (the
    network of Sec. "Training based on dissipation rates")."""
    rng = _rng(31)
    f = inputs.random_populations((6,), seed=32, lo=0.8, hi=1.2)
    lam = rng.standard_normal((27, 6))
    layers = collision.unpack_params(inputs.mlp_params(8, 33, depth=3), 8, depth=3)
    assert len(layers) == 4
    tau, h = 0.56, 1e-6
    g_f, g_p = adjoint.nco_collide_vjp(f, lam, tau, layers, "tanh")
    d = rng.standard_normal((27, 6))
    fd = ((collision.nco(f + h * d, tau, layers) - collision.nco(f - h * d, tau, layers)) / (2 * h) * lam).sum()
    assert abs(fd - (g_f * d).sum()) < 1e-7 * max(1.0, abs(fd))
    v = rng.standard_normal(collision.n_params(8, depth=3))
    fd = ((collision.nco(f, tau, _perturb(layers, v, h)) - collision.nco(f, tau, _perturb(layers, v, -h)))
          / (2 * h) * lam).sum()
    assert abs(fd - adjoint.flatten(g_p) @ v) < 1e-7 * max(1.0, abs(fd))


def test_force_vjp_matches_finite_differences():
    """dL/dF of one forced collision, L = <w, x_next>, against central
    differences in the force."""
    rng = _rng(90)
    n, tau = 4, 0.56
    layers = _layers(8, 91)
    f = inputs.random_populations((n, n, n), seed=92, lo=0.9, hi=1.1)
    F = 1e-3 * rng.standard_normal((3, n, n, n))
    w = rng.standard_normal(f.shape)
    op = step.Operator("nco", tau, layers=layers, act="tanh")
    y = step.stream(f).reshape(27, -1)
    g = adjoint.force_vjp(y.sum(0), adjoint._C.T @ y, F.reshape(3, -1), w.reshape(27, -1))
    h = 1e-6
    for _ in range(2):
        d = rng.standard_normal(F.shape)
        fd = ((w * step.step(f, op, F + h * d)).sum() - (w * step.step(f, op, F - h * d)).sum()) / (2 * h)
        an = (g * d.reshape(3, -1)).sum()
        assert abs(fd - an) < 1e-7 * abs(an), (fd, an)


def test_unrolled_gradient_with_velocity_dependent_phase():
    """Alvelius' rule makes each step's force a function of the state it
    starts from; the reverse mode through it matches central differences of
    the forward run (parameters and initial populations), and dropping that
    path (the same forces held fixed) gives a visibly different gradient."""
    n, width, tau, T = 6, 8, 0.55, 3
    rng = _rng(93)
    layers = _layers(width, 94)
    _, u = inputs.turbulence(n, seed=95, k0=2.0, urms=0.05)
    f0 = collision.equilibrium(np.ones((n, n, n)), u)
    ks = inputs.forcing_half_modes(2.0)
    draws = inputs.uniform_draws(T, len(ks), 96)
    sf = (ks, draws, 1e-4, 1.5, 1.0)
    w = rng.standard_normal(f0.shape)

    def loss_grad(x):
        return float((w * x).sum()), w

    def forward(lay, g0):
        op = step.Operator("nco", tau, layers=lay, act="tanh")
        x, fields = g0, []
        for t in range(T):
            _, ut = collision.macroscopic(x)
            fields.append(forcing.field(ks, forcing.coefficients_state(ks, draws[t], 1e-4, 1.5, 1.0, ut), (n, n, n)))
            x = step.step(x, op, fields[-1])
        return float((w * x).sum()), fields
    L, gp, gf0 = adjoint.run_and_grad(f0, tau, layers, "tanh", T, loss_grad, state_forcing=sf)
    L0, fields = forward(layers, f0)
    assert abs(L - L0) < 1e-12 * abs(L0)
    h = 1e-6
    v = rng.standard_normal(collision.n_params(width))
    fd = (forward(_perturb(layers, v, h), f0)[0] - forward(_perturb(layers, v, -h), f0)[0]) / (2 * h)
    an = adjoint.flatten(gp) @ v
    assert abs(fd - an) < 1e-6 * abs(an), (fd, an)
    d = 1e-3 * rng.standard_normal(f0.shape)
    fd = (forward(layers, f0 + h * d)[0] - forward(layers, f0 - h * d)[0]) / (2 * h)
    an = (gf0 * d).sum()
    assert abs(fd - an) < 1e-6 * abs(an), (fd, an)
    # Negative control: the forces of this run held fixed.
    _, _, frozen = adjoint.run_and_grad(f0, tau, layers, "tanh", T, loss_grad, forces=lambda t: fields[t])
    assert abs((frozen * d).sum() - an) > 1e3 * abs(fd - an)
