"""GPU forcing and reverse mode against the float64 oracle, through the C ABI.

The GPU gradient is float32 arithmetic; it is compared with the oracle's
float64 gradient of the same run in relative 2-norm."""
import numpy as np
import pytest

from oracle import adjoint, collision, forcing, observables, step
from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L
from paper_2412_08229_amd.training import log_spectrum_loss

pytestmark = pytest.mark.gpu

AMP, KF, CW = 2e-6, 1.5, 1.0


def _forcing(n_steps, seed):
    ks = inputs.forcing_half_modes(2.0)
    draws = inputs.uniform_draws(n_steps, len(ks), seed)
    return ks, draws


def _oracle_forces(ks, draws, shape):
    fh = forcing.coefficients(ks, draws, AMP, KF, CW)
    return lambda t: forcing.field(ks, fh[t % len(fh)], shape)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_forced_steps_match_oracle(storage, tol):
    n, T = 8, 5
    ks, draws = _forcing(3, seed=1)
    f0 = inputs.random_populations((n, n, n), seed=2, lo=0.9, hi=1.1)
    with Lattice((n, n, n), storage, "bgk", 0.6) as lat:
        lat.set_forcing(ks, draws, AMP, KF, CW)
        lat.init_populations(f0)
        fs = lat.populations()
        lat.step(T)
        got = lat.populations()
    want = step.run(fs, step.Operator("bgk", 0.6), T, forces=_oracle_forces(ks, draws, (n, n, n)))
    assert np.abs(got - want).max() < tol


# Power-input forcing: every integer wavevector of the band 0.5 <= |k| <= 2.5
# (40 of each +-k pair), Gaussian peak 1.5, width 1, power in lattice units.
PK_A, PK_B, P_IN = 0.5, 2.5, 1e-6


@pytest.mark.parametrize("shape,storage,kind,mlp,tol", [((12, 12, 12), "f64", "bgk", "f32", 1e-13),
                                                        ((12, 12, 12), "f32", "nco", "f32_mfma", 2e-6),
                                                        ((11, 13, 10), "f64", "nco", "f32", 1e-13)])
def test_power_input_forcing_matches_oracle(shape, storage, kind, mlp, tol):
    """nco_set_forcing_power: the amplitude from the power input (the
    equation for A, Sec. "Training Data - Forced Isotropic Turbulence") and
    the forced steps, drawn phases and the velocity-dependent phase, against
    the oracle's amplitude_from_power and forced steps."""
    T = 4
    ks = inputs.forcing_half_modes(PK_B, PK_A)
    draws = inputs.uniform_draws(3, len(ks), seed=101)
    amp = forcing.amplitude_from_power(P_IN, 1.0, PK_A, PK_B, KF, CW)
    assert abs(L.nco_forcing_amplitude(P_IN, 1.0, PK_A, PK_B, KF, CW) / amp - 1) < 1e-12
    _, u = inputs.random_velocity(shape, seed=102, amp=0.05)
    rho = np.ones(shape)
    params = inputs.mlp_params(32, 103)
    op = step.Operator(kind, 0.6, layers=collision.unpack_params(params, 32), act="tanh")
    for rule in (False, True):
        with Lattice(shape, storage, kind, 0.6) as lat:
            if kind == "nco":
                lat.set_net_weights(params, 32, "tanh", mlp)
            lat.set_forcing_power(ks, draws, P_IN, PK_A, PK_B, KF, CW, phase_rule=rule)
            lat.init_equilibrium(rho, u)
            f = lat.populations()
            lat.step(T)
            got = lat.populations()
        fh = forcing.coefficients(ks, draws, amp, KF, CW)
        for t in range(T):
            if rule:
                _, ut = collision.macroscopic(f)
                coef = forcing.coefficients_state(ks, draws[t % 3], amp, KF, CW, ut)
            else:
                coef = fh[t % 3]
            f = step.step(f, op, force=forcing.field(ks, coef, shape))
        err = np.abs(got - f).max()
        print("power forcing %s %s/%s rule=%s: max err %.3e" % (shape, storage, mlp, rule, err))
        assert err < tol


@pytest.mark.parametrize("rule", [False, True])
def test_gradient_matches_oracle_at_the_training_form(rule):
    """The reverse mode at the form of the forced-turbulence training, scaled
    to what the oracle finishes in seconds: 16^3, 20 steps in checkpoint
    segments of 5, forcing from the power input (drawn phases, or the
    velocity-dependent phase with the gradient through it), the log-spectrum
    loss over 2 <= k <= 6.  dL/dtheta and dL/df0 of the float32 GPU adjoint
    (vector-unit and matrix-core networks) within 1e-3 of the oracle's
    float64 reverse mode."""
    n, width, tau, T, K, kmin, kmax = 16, 32, 0.52, 20, 5, 2, 6
    params = inputs.mlp_params(width, 104)
    _, u = inputs.turbulence(n, seed=105, k0=4.0, urms=0.05)
    rho = np.ones((n, n, n))
    f_init = collision.equilibrium(rho, u)
    Et = observables.spectrum(f_init) * np.linspace(0.8, 1.2, observables.n_bins(n)) + 1e-12
    ks = inputs.forcing_half_modes(PK_B, PK_A)
    draws = inputs.uniform_draws(T, len(ks), seed=106)
    amp = forcing.amplitude_from_power(P_IN, 1.0, PK_A, PK_B, KF, CW)
    layers = collision.unpack_params(params, width)

    def loss_grad(x):
        Lx, d = adjoint.log_spectrum_loss(observables.spectrum(x), Et, kmin, kmax)
        return Lx, adjoint.spectrum_vjp(x, d)
    if rule:
        Lo, go, gfo = adjoint.run_and_grad(f_init, tau, layers, "tanh", T, loss_grad,
                                           state_forcing=(ks, draws, amp, KF, CW))
    else:
        fh = forcing.coefficients(ks, draws, amp, KF, CW)
        Lo, go, gfo = adjoint.run_and_grad(f_init, tau, layers, "tanh", T, loss_grad,
                                           forces=lambda t: forcing.field(ks, fh[t], (n, n, n)))
    go = adjoint.flatten(go)
    for mlp in ("f32_mfma", "f32"):
        with Lattice((n, n, n), "f32", "nco", tau) as lat:
            lat.set_net_weights(params, width, "tanh", mlp)
            lat.set_forcing_power(ks, draws, P_IN, PK_A, PK_B, KF, CW, phase_rule=rule)
            lat.init_populations(f_init)
            lat.forward_record(T, K)
            Lg, dE = log_spectrum_loss(lat.energy_spectrum(), Et, kmin, kmax)
            g, df0 = lat.backward(dL_dE=dE, want_df0=True)
        rel = np.linalg.norm(g - go) / np.linalg.norm(go)
        relf = np.linalg.norm(df0 - gfo) / np.linalg.norm(gfo)
        print("16^3 x %d (K=%d) rule=%s %s: loss %.8e vs %.8e, dL/dtheta rel err %.2e, dL/df0 rel err %.2e"
              % (T, K, rule, mlp, Lg, Lo, rel, relf))
        assert abs(Lg - Lo) < 1e-4 * abs(Lo)
        assert rel < 1e-3 and relf < 1e-3


def _setup(n, width, seed, act):
    params = inputs.mlp_params(width, seed)
    _, u = inputs.turbulence(n, seed=seed + 1, k0=2.0, urms=0.04)
    rho = np.ones((n, n, n))
    f0 = collision.equilibrium(rho, u)
    Et = observables.spectrum(f0) * np.linspace(0.7, 1.3, observables.n_bins(n)) + 1e-12
    return params, rho, u, f0, Et


@pytest.mark.parametrize("act,mlp,forced", [("tanh", "f32", False), ("tanh", "f32_mfma", True),
                                            ("relu", "f32", False), ("tanh", "f32_mfma", False),
                                            ("relu", "f32_mfma", True),
                                            # split products in the recorded and recomputed steps,
                                            # the float32 matrix-core adjoint behind them
                                            ("tanh", "f32_split", True), ("relu", "f32_split", False)])
def test_spectrum_loss_gradient_matches_oracle(act, mlp, forced):
    n, width, tau, T, K = 8, 32, 0.56, 6, 4
    params, rho, u, f0, Et = _setup(n, width, 4, act)
    ks, draws = _forcing(T, seed=5)
    kmin, kmax = 1, 3
    with Lattice((n, n, n), "f32", "nco", tau) as lat:
        lat.set_net_weights(params, width, act, mlp)
        if forced:
            lat.set_forcing(ks, draws, AMP, KF, CW)
        lat.init_equilibrium(rho, u)
        fs = lat.populations()
        lat.forward_record(T, K)
        E = lat.energy_spectrum()
        Lg, dE = log_spectrum_loss(E, Et, kmin, kmax)
        g, df0 = lat.backward(dL_dE=dE, want_df0=True)
    layers = collision.unpack_params(params, width)
    forces = _oracle_forces(ks, draws, (n, n, n)) if forced else None

    def loss_grad(x):
        Lx, d = adjoint.log_spectrum_loss(observables.spectrum(x), Et, kmin, kmax)
        return Lx, adjoint.spectrum_vjp(x, d)
    Lo, go, gfo = adjoint.run_and_grad(fs, tau, layers, act, T, loss_grad, forces=forces)
    go = adjoint.flatten(go)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    relf = np.linalg.norm(df0 - gfo) / np.linalg.norm(gfo)
    print("%s/%s forced=%s: loss %.6e vs %.6e, grad rel err %.2e, dL/df0 rel err %.2e"
          % (act, mlp, forced, Lg, Lo, rel, relf))
    assert abs(Lg - Lo) < 1e-4 * abs(Lo)
    assert rel < 2e-3 and relf < 2e-3


def test_spectrum_loss_gradient_matches_oracle_above_64():
    """The spectrum and its reverse mode on a 66^3 lattice: the complex DFT
    passes take two 64-frequency groups per lane above 64, with a ragged
    frequency block (66 of 128) and a ragged last block of lines; the readout
    transforms the half spectrum, the reverse mode the full one.  Two steps
    (the collision keeps the velocity, so the spectrum of one step does not
    depend on the network) of the 27-8-8-8-4 tanh network (depth 3,
    matrix-core forward) keep the oracle's run short."""
    n, width, tau, kmin, kmax = 66, 8, 0.56, 2, 12
    params = inputs.mlp_params(width, 4, depth=3)
    _, u = inputs.turbulence(n, seed=5, k0=4.0, urms=0.04)
    f0 = collision.equilibrium(np.ones((n, n, n)), u)
    Et = observables.spectrum(f0) * np.linspace(0.7, 1.3, observables.n_bins(n)) + 1e-12
    with Lattice((n, n, n), "f32", "nco", tau) as lat:
        lat.set_net_weights(params, width, "tanh", "f32_mfma", depth=3)
        lat.init_populations(f0)
        lat.forward_record(2, 1)
        E = lat.energy_spectrum()
        f2 = lat.populations()
        Lg, dE = log_spectrum_loss(E, Et, kmin, kmax)
        g, df0 = lat.backward(dL_dE=dE, want_df0=True)
    np.testing.assert_allclose(E, observables.spectrum(f2.astype(np.float64)), rtol=1e-11, atol=1e-18)
    layers = collision.unpack_params(params, width, depth=3)

    def loss_grad(x):
        Lx, d = adjoint.log_spectrum_loss(observables.spectrum(x), Et, kmin, kmax)
        return Lx, adjoint.spectrum_vjp(x, d)
    Lo, go, gfo = adjoint.run_and_grad(f0, tau, layers, "tanh", 2, loss_grad)
    go = adjoint.flatten(go)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    relf = np.linalg.norm(df0 - gfo) / np.linalg.norm(gfo)
    print("66^3 x 2: loss %.8e vs %.8e, grad rel err %.2e, dL/df0 rel err %.2e" % (Lg, Lo, rel, relf))
    assert abs(Lg - Lo) < 1e-4 * abs(Lo)
    assert rel < 2e-3 and relf < 2e-3


@pytest.mark.parametrize("n", [48, 129])
def test_spectrum_reverse_mode_through_one_step_at_size(n):
    """A property that holds at any size: the collision keeps rho and j, and
    a dL/dx that depends on rho and j only passes its adjoint unchanged (the
    rates act on non-conserved moments only), so after one step the gradient
    of a spectrum loss with respect to the start is the streaming's adjoint of
    the spectrum's reverse mode, dL/df0 = unstream(spectrum_vjp(x_1, dL/dE)).
    48^3 takes one 64-frequency group per lane, 129^3 four (odd: no Nyquist
    shell, ragged blocks of lines and frequencies); the readout E(k) of x_1
    is checked against the oracle on the way."""
    _, u = inputs.turbulence(n, seed=11, k0=4.0, urms=0.04)
    with Lattice((n, n, n), "f32", "nco", 0.56) as lat:
        lat.set_net_weights(inputs.mlp_params(32, 9), 32, "tanh", "f32_mfma")
        lat.init_equilibrium(None, u)
        lat.forward_record(1, 1)
        E = lat.energy_spectrum()
        f1 = lat.populations().astype(np.float64)
        Et = E * np.linspace(0.8, 1.2, len(E)) + 1e-12
        _, dE = log_spectrum_loss(E, Et, 2, n // 3)
        _, df0 = lat.backward(dL_dE=dE, want_df0=True)
    np.testing.assert_allclose(E, observables.spectrum(f1), rtol=1e-11, atol=1e-18)
    want = step.unstream(adjoint.spectrum_vjp(f1, dE))
    rel = np.linalg.norm(df0 - want) / np.linalg.norm(want)
    print("%d^3: dL/df0 through one step vs unstream(spectrum_vjp), rel err %.2e" % (n, rel))
    assert rel < 2e-5


@pytest.mark.parametrize("shape,mlp", [((6, 6, 6), "f32"), ((6, 6, 6), "f32_mfma"), ((7, 6, 9), "f32_mfma"),
                                       ((3, 11, 17), "f32_mfma")])
def test_population_loss_gradient_and_determinism(shape, mlp):
    """Loss <w, x_T> given as dL/df; two backward passes agree bitwise.  The
    lattices with 378 and 561 nodes end in a partial block of the
    matrix-core adjoint."""
    width, tau, T, K = 32, 0.57, 5, 2
    params = inputs.mlp_params(width, 7)
    f0 = inputs.random_populations(shape, seed=8, lo=0.95, hi=1.05)
    w = np.random.Generator(np.random.PCG64(9)).standard_normal(f0.shape)
    grads = []
    with Lattice(shape, "f32", "nco", tau) as lat:
        lat.set_net_weights(params, width, "tanh", mlp)
        for _ in range(2):
            lat.init_populations(f0)
            fs = lat.populations()
            lat.forward_record(T, K)
            grads.append(lat.backward(dL_df=w, want_df0=True))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
    layers = collision.unpack_params(params, width)
    _, go, gfo = adjoint.run_and_grad(fs, tau, layers, "tanh", T, lambda x: (float((w * x).sum()), w))
    go = adjoint.flatten(go)
    assert np.linalg.norm(grads[0][0] - go) / np.linalg.norm(go) < 2e-3
    assert np.linalg.norm(grads[0][1] - gfo) / np.linalg.norm(gfo) < 1e-4


def test_backward_state_errors():
    with Lattice((4, 4, 4), "f32", "nco", 0.6) as lat:
        lat.set_net_weights(inputs.mlp_params(32, 0), 32)
        with pytest.raises(L.NCOError) as e:
            lat.backward(dL_df=np.zeros((27, 4, 4, 4)))
        assert e.value.status == L.NCO_E_STATE
        lat.forward_record(3, 2)
        lat.step(1)
        with pytest.raises(L.NCOError) as e:
            lat.backward(dL_df=np.zeros((27, 4, 4, 4)))
        assert e.value.status == L.NCO_E_STATE
    with Lattice((4, 4, 4), "f32", "nco", 0.6) as lat:
        lat.set_net_weights(inputs.mlp_params(16, 0), 16)
        with pytest.raises(L.NCOError) as e:
            lat.forward_record(3, 2)
        assert e.value.status == L.NCO_E_UNSUPPORTED


def test_bf16_network_gradient_close_to_float32():
    """A bf16 network runs its forward in bf16 and its reverse mode in
    float32: the gradient stays within bf16 rounding of the float32
    network's."""
    n, width, tau, T, K = 8, 32, 0.56, 6, 3
    params, rho, u, f0, Et = _setup(n, width, 4, "tanh")
    out = {}
    for mlp in ("f32_mfma", "bf16"):
        with Lattice((n, n, n), "f32", "nco", tau) as lat:
            lat.set_net_weights(params, width, "tanh", mlp)
            lat.init_equilibrium(rho, u)
            lat.forward_record(T, K)
            _, dE = log_spectrum_loss(lat.energy_spectrum(), Et, 1, 3)
            out[mlp] = lat.backward(dL_dE=dE)[0]
    rel = np.linalg.norm(out["bf16"] - out["f32_mfma"]) / np.linalg.norm(out["f32_mfma"])
    print("bf16 vs float32 network gradient: rel %.2e" % rel)
    assert rel < 5e-2


@pytest.mark.parametrize("mlp", ["f32", "f32_mfma"])
def test_energy_trajectory_gradient_matches_oracle(mlp):
    """Loss on the kinetic-energy trajectory (states t = 0, 2, 4, 6 of a
    6-step run, checkpoints every 4): the recorded samples match the
    oracle's k(t), and the gradient of sum_m a_m k(t_m) matches the oracle's
    reverse mode with the same intermediate terms."""
    n, width, tau, T, K, every = 8, 32, 0.56, 6, 4, 2
    params = inputs.mlp_params(width, 21)
    rho, u = inputs.random_velocity((n, n, n), seed=22, amp=0.08)
    a = np.random.Generator(np.random.PCG64(23)).standard_normal(T // every + 1)
    with Lattice((n, n, n), "f32", "nco", tau) as lat:
        lat.set_net_weights(params, width, "tanh", mlp)
        lat.init_equilibrium(rho, u)
        fs = lat.populations()
        k = lat.forward_record(T, K, energy_every=every)
        g, df0 = lat.backward(dL_dk=a, energy_every=every, want_df0=True)
    layers = collision.unpack_params(params, width)
    op = step.Operator("nco", tau, layers=layers, act="tanh")
    x, k_o = fs, [observables.kinetic_energy(fs)]
    for t in range(1, T + 1):
        x = step.step(x, op)
        if t % every == 0:
            k_o.append(observables.kinetic_energy(x))
    assert np.abs(k - np.array(k_o)).max() < 1e-6 * max(k_o)

    def traj(t, xt):
        return a[t // every] * adjoint.kinetic_energy_vjp(xt) if t % every == 0 else None
    _, go, gfo = adjoint.run_and_grad(fs, tau, layers, "tanh", T, lambda xt: (0.0, np.zeros_like(xt)),
                                      traj_grad=traj)
    go = adjoint.flatten(go)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    relf = np.linalg.norm(df0 - gfo) / np.linalg.norm(gfo)
    print("energy trajectory %s: grad rel err %.2e, dL/df0 rel err %.2e" % (mlp, rel, relf))
    assert rel < 2e-3 and relf < 2e-3


@pytest.mark.parametrize("shape,storage,kind,mlp,tol", [((12, 12, 12), "f64", "bgk", "f32", 1e-13),
                                                        ((12, 12, 12), "f64", "nco", "f32", 1e-13),
                                                        ((12, 12, 12), "f32", "nco", "f32_mfma", 2e-6),
                                                        ((17, 13, 11), "f64", "bgk", "f32", 1e-13)])
def test_velocity_dependent_phase_matches_oracle(shape, storage, kind, mlp, tol):
    """Alvelius' velocity-dependent theta1 (nco_set_forcing_ex): each step's
    coefficients come from the velocity of the state it starts from; the
    GPU run equals the oracle's (coefficients_state, then the forced step)
    on a 12^3 lattice (ragged against the 256-node blocks) and a 17x13x11
    one (2431 nodes: two blocks of the 2048-node mode sums, the second
    partial), and differs from the run with the drawn theta1."""
    T, amp = 5, 1e-4
    ks, draws = _forcing(4, seed=61)
    if len(set(shape)) == 1:
        _, u = inputs.turbulence(shape[0], seed=62, k0=2.0, urms=0.05)
    else:
        _, u = inputs.random_velocity(shape, seed=62, amp=0.05)
    rho = np.ones(shape)
    params = inputs.mlp_params(32, 63)
    layers = collision.unpack_params(params, 32)
    runs = {}
    for rule in (True, False):
        with Lattice(shape, storage, kind, 0.6) as lat:
            if kind == "nco":
                lat.set_net_weights(params, 32, "tanh", mlp)
            lat.set_forcing(ks, draws, amp, KF, CW, phase_rule=rule)
            lat.init_equilibrium(rho, u)
            f0 = lat.populations()
            lat.step(T)
            runs[rule] = lat.populations()
    op = step.Operator(kind, 0.6, layers=layers, act="tanh")
    f = f0
    for t in range(T):
        _, ut = collision.macroscopic(f)
        fh = forcing.coefficients_state(ks, draws[t % len(draws)], amp, KF, CW, ut)
        f = step.step(f, op, force=forcing.field(ks, fh, shape))
    err = np.abs(runs[True] - f).max()
    print("phase rule %s/%s/%s: max err %.3e, vs drawn phase %.3e"
          % (storage, kind, mlp, err, np.abs(runs[True] - runs[False]).max()))
    assert err < tol
    assert np.abs(runs[True] - runs[False]).max() > 100 * tol


@pytest.mark.parametrize("shape,mlp,loss", [((8, 8, 8), "f32_mfma", "population"), ((7, 6, 9), "f32", "population"),
                                             ((8, 8, 8), "f32_mfma", "spectrum"), ((9, 9, 9), "f32", "spectrum"),
                                             ((13, 14, 15), "f32_mfma", "population")])
def test_velocity_dependent_phase_gradient_matches_oracle(shape, mlp, loss):
    """Reverse mode through Alvelius' velocity-dependent theta1: the force of
    each step depends on the state it starts from, and the GPU gradient
    (parameters and dL/df0) follows that path like the oracle's.  The
    recording starts 2 steps into a forcing period of 3 draws and spans 5
    steps in checkpoint segments of 2 (the recomputed segments replay the
    kept coefficients); the lattices of 378 and 729 nodes end in a partial
    block, and the one of 2730 nodes spans two blocks of the 1024-node mode
    sums of the reverse pass, the second partial.  Two backward passes agree bitwise, and the gradient with the same
    forces held fixed is far from both."""
    width, tau, T, K, amp, t0 = 32, 0.58, 5, 2, 1e-4, 2
    n_nodes = int(np.prod(shape))
    ks, draws = _forcing(3, seed=67)
    params = inputs.mlp_params(width, 68)
    if len(set(shape)) == 1:
        _, u = inputs.turbulence(shape[0], seed=69, k0=2.0, urms=0.05)
    else:
        _, u = inputs.random_velocity(shape, seed=69, amp=0.05)
    rho = np.ones(shape)
    f_init = collision.equilibrium(rho, u)
    w = np.random.Generator(np.random.PCG64(70)).standard_normal((27,) + shape)
    Et = None
    if loss == "spectrum":
        Et = observables.spectrum(f_init) * np.linspace(0.7, 1.3, observables.n_bins(shape[0])) + 1e-12
    grads = []
    with Lattice(shape, "f32", "nco", tau) as lat:
        lat.set_net_weights(params, width, "tanh", mlp)
        lat.set_forcing(ks, draws, amp, KF, CW, phase_rule=True)
        lat.init_equilibrium(rho, u)
        lat.step(t0)                                   # forcing step t0 next
        for _ in range(2):
            lat.init_populations(f_init)
            fs = lat.populations()
            lat.forward_record(T, K)
            if loss == "spectrum":
                _, dE = log_spectrum_loss(lat.energy_spectrum(), Et, 1, 3)
                grads.append(lat.backward(dL_dE=dE, want_df0=True))
            else:
                grads.append(lat.backward(dL_df=w, want_df0=True))
            lat.step(3 - T % 3)                         # back to forcing step t0
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
    g, df0 = grads[0]
    layers = collision.unpack_params(params, width)
    rolled = np.roll(draws, -t0, axis=0)
    sf = (ks, rolled, amp, KF, CW)

    if loss == "spectrum":
        def loss_grad(x):
            Lx, d = adjoint.log_spectrum_loss(observables.spectrum(x), Et, 1, 3)
            return Lx, adjoint.spectrum_vjp(x, d)
    else:
        def loss_grad(x):
            return float((w * x).sum()), w
    _, go, gfo = adjoint.run_and_grad(fs, tau, layers, "tanh", T, loss_grad, state_forcing=sf)
    go = adjoint.flatten(go)
    # The same run with its forces held fixed: the reverse mode without the phase path.
    op = step.Operator("nco", tau, layers=layers, act="tanh")
    x, fields = fs, []
    for t in range(T):
        _, ut = collision.macroscopic(x)
        fields.append(forcing.field(ks, forcing.coefficients_state(ks, rolled[t % 3], amp, KF, CW, ut), shape))
        x = step.step(x, op, fields[-1])
    _, gz, gfz = adjoint.run_and_grad(fs, tau, layers, "tanh", T, loss_grad, forces=lambda t: fields[t])
    gz = adjoint.flatten(gz)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    relf = np.linalg.norm(df0 - gfo) / np.linalg.norm(gfo)
    relz = np.linalg.norm(gfz - gfo) / np.linalg.norm(gfo)
    print("phase-rule gradient %s %s %s (%d nodes): grad rel err %.2e, dL/df0 rel err %.2e; frozen-force "
          "dL/df0 differs by %.2e" % (shape, mlp, loss, n_nodes, rel, relf, relz))
    # float32 adjoint arithmetic over 5 steps and < 1000 nodes: measured
    # errors stay below 1e-5.
    assert rel < 1e-4 and relf < 1e-4
    assert relz > 100 * relf


def test_velocity_dependent_phase_refused_by_batched_steps():
    n = 8
    ks, draws = _forcing(2, seed=64)
    _, u = inputs.turbulence(n, seed=65, k0=2.0, urms=0.05)
    with Lattice((n, n, n), "f32", "nco", 0.6) as lat:
        lat.set_net_weights(inputs.mlp_params(32, 66), 32, "tanh", "f32_mfma")
        lat.set_forcing(ks, draws, 1e-4, KF, CW, phase_rule=True)
        lat.init_equilibrium(None, u)
        from paper_2412_08229_amd.lattice import batch_step
        with pytest.raises(L.NCOError) as e:
            batch_step([lat], [2])
        assert e.value.status == L.NCO_E_UNSUPPORTED
        lat.forward_record(4, 2)




@pytest.mark.parametrize("n", [32, 48, 64])
def test_vector_adjoint_matches_matrix_core_adjoint_at_size(n):
    """The vector-unit adjoint splits each 64-node block's group elements
    over four wavefronts up to 2048 blocks and keeps one wavefront above; the
    matrix-core adjoint runs 64-node blocks (one tile per wavefront) below
    65536 nodes and 256-node blocks above.  Across these switches (32^3: 512
    and 512 blocks, 48^3: 1728 and 432, 64^3: 4096 and 1024) the two
    gradients agree on the same recorded 12-step run to float32 accumulation
    error; both are pinned to the oracle at small sizes.  The loss
    weights have random signs, so the parameter gradient is a sum with heavy
    cancellation: both paths differ from each other by ~1e-6 absolute at
    16^3 .. 64^3, a few 1e-4 of the gradient's norm where that norm is small
    (2.6e-3 at 48^3, 1.1e-2 at 64^3)."""
    width, tau, T, K = 32, 0.56, 12, 4
    params = inputs.mlp_params(width, 71)
    _, u = inputs.turbulence(n, seed=72, k0=4.0, urms=0.05)
    w = np.random.Generator(np.random.PCG64(73)).standard_normal((27, n, n, n))
    out = {}
    for mlp in ("f32", "f32_mfma"):
        with Lattice((n, n, n), "f32", "nco", tau) as lat:
            lat.set_net_weights(params, width, "tanh", mlp)
            lat.init_equilibrium(None, u)
            lat.forward_record(T, K)
            out[mlp] = lat.backward(dL_df=w, want_df0=True)
    rel = np.linalg.norm(out["f32"][0] - out["f32_mfma"][0]) / np.linalg.norm(out["f32_mfma"][0])
    relf = np.linalg.norm(out["f32"][1] - out["f32_mfma"][1]) / np.linalg.norm(out["f32_mfma"][1])
    print("%d^3: vector vs matrix-core adjoint, grad rel diff %.2e, dL/df0 rel diff %.2e" % (n, rel, relf))
    assert rel < 1e-3 and relf < 1e-5


@pytest.mark.parametrize("n,forced,K", [(24, False, 5), (48, True, 5), (24, True, 1)])
def test_reverse_cache_leaves_the_gradient_unchanged(n, forced, K):
    """The recomputed forward steps of a segment keep their network values
    (group sums, tilde tau), the recorded run keeps those of the last state
    of each segment, and the matrix-core adjoint reads them instead of
    running the network again: the same arithmetic on the same states, so
    the gradient must not change at all, whether nothing, only the
    recompute's share or everything fits the budget.  24^3 runs the 64-node
    kernels, 48^3 the 256-node ones; 12 steps with checkpoints every 5 give
    segments of 5, 5 and 2 states, with checkpoints every step 12 of 1."""
    width, tau, T = 32, 0.56, 12
    params = inputs.mlp_params(width, 81)
    _, u = inputs.turbulence(n, seed=82, k0=4.0, urms=0.05)
    w = np.random.Generator(np.random.PCG64(83)).standard_normal((27, n, n, n))
    state_bytes = -(-n ** 3 // 256) * 256 * 36 * 4
    out = []
    for cache in (0, (K - 1) * state_bytes + 1, 1 << 30):
        with Lattice((n, n, n), "f32", "nco", tau) as lat:
            lat.set_net_weights(params, width, "tanh", "f32_mfma")
            lat.set_reverse_cache(cache)
            if forced:
                ks, draws = _forcing(T, seed=84)
                lat.set_forcing(ks, draws, AMP, KF, CW)
            lat.init_equilibrium(None, u)
            lat.forward_record(T, K)
            out.append(lat.backward(dL_df=w, want_df0=True))
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0])
        assert np.array_equal(out[0][1], o[1])
